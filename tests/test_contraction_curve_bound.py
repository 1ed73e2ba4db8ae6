"""The bound that lets the march skip along contracted rays (Sec. 4, the
L-infinity contraction): over a stretch [t_a, t_b] of a straight ray whose
two ends have the same dominant axis i, with the same sign and |u_i| > 1,
the contracted image C(o + t d) stays inside the box spanned by
  axis i:      sign * [min, max] of (2 - 1/|u_i|) at the two ends,
  other axes:  [min, max] of the four products a * b, with a = 2 - 1/|u_i|
               and b = u_j / |u_i| taken at the two ends.
The GPU march uses this box, padded by a hundredth of a cell, both to walk
runs of clear coarse blocks and to skip single empty boxes beyond the unit
ball.  Here the argument is checked in FP64 on densely sampled curves of
seeded random rays, and checked to be tight enough to be useful (it does not
degenerate to the whole cube).  CPU only; no GPU code is involved."""
import numpy as np


def contract(u):
    m = np.max(np.abs(u), axis=-1, keepdims=True)
    return np.where(m <= 1.0, u, (2.0 - 1.0 / m) * u / m)


def end_box(ua, ub):
    """The box of the argument from the two end points (None if it does not apply)."""
    ia, ib = int(np.argmax(np.abs(ua))), int(np.argmax(np.abs(ub)))
    ma, mb = np.abs(ua[ia]), np.abs(ub[ib])
    if ia != ib or np.sign(ua[ia]) != np.sign(ub[ib]) or not (ma > 1.0 and mb > 1.0):
        return None
    aa, ab = 2.0 - 1.0 / ma, 2.0 - 1.0 / mb
    alo, ahi = min(aa, ab), max(aa, ab)
    lo, hi = np.empty(3), np.empty(3)
    for a in range(3):
        if a == ia:
            s = np.sign(ua[ia])
            lo[a], hi[a] = (alo, ahi) if s > 0 else (-ahi, -alo)
        else:
            b = (ua[a] / ma, ub[a] / mb)
            p = [x * y for x in (alo, ahi) for y in (min(b), max(b))]
            lo[a], hi[a] = min(p), max(p)
    return lo, hi


def test_curve_stays_in_end_box():
    rng = np.random.default_rng(20231105)
    checked = 0
    widths = []
    for _ in range(4000):
        o = rng.uniform(-1.5, 1.5, 3)
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        ta = rng.uniform(0.0, 8.0)
        tb = ta + rng.exponential(0.5)
        ua, ub = o + ta * d, o + tb * d
        box = end_box(ua, ub)
        if box is None:
            continue
        lo, hi = box
        t = np.linspace(ta, tb, 257)
        y = contract(o[None, :] + t[:, None] * d[None, :])
        assert np.all(y >= lo - 1e-12) and np.all(y <= hi + 1e-12), (o, d, ta, tb)
        widths.append(np.max(hi - lo) / max(np.max(y.max(0) - y.min(0)), 1e-12))
        checked += 1
    assert checked > 1000
    # tight: the box is no wider than a few times the curve's own extent
    assert np.median(widths) < 2.0


def test_bound_refuses_mixed_stretches():
    """The argument needs the same dominant axis and sign at both ends, and
    both ends outside the unit ball; otherwise no box is claimed."""
    assert end_box(np.array([1.5, 0.2, 0.1]), np.array([0.2, 1.6, 0.0])) is None   # axis changes
    assert end_box(np.array([1.5, 0.2, 0.1]), np.array([-1.7, 0.2, 0.1])) is None  # sign changes
    assert end_box(np.array([0.9, 0.2, 0.1]), np.array([1.7, 0.2, 0.1])) is None   # start inside the ball
    assert end_box(np.array([1.2, 0.2, 0.1]), np.array([3.0, -0.5, 0.4])) is not None


def test_box_is_exact_on_axis_rays():
    """A ray along +x from inside the shell: y_x runs over [2 - 1/|u_a|, 2 - 1/|u_b|]
    and the other coordinates stay 0."""
    ua, ub = np.array([1.25, 0.0, 0.0]), np.array([4.0, 0.0, 0.0])
    lo, hi = end_box(ua, ub)
    assert np.allclose(lo, [2 - 1 / 1.25, 0.0, 0.0]) and np.allclose(hi, [2 - 1 / 4.0, 0.0, 0.0])
