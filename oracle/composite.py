"""Front-to-back alpha compositing with early termination, FP64.

Volume rendering as NeRF/iNGP do it (the paper composites PQ colors and
matches them to PQ images, Sec. 4.1 and App. C): for the evaluated samples
of a ray in increasing t, with step delta = dt for every sample,
    alpha_j = 1 - exp(-sigma_j delta),  C += T alpha_j c_j,  T <- T (1 - alpha_j).
Background 0; output (C_rgb, A = 1 - T, number of composited samples).

Early termination (not in the paper; the workloads ask for it): stop after
the sample that makes T < t_min.  Because an FP32 renderer may decide
T < t_min differently from FP64 when T is within rounding of t_min, the
oracle also reports the two ends of the range of acceptable stopping points:
"lo" = first j with T < t_min (1 + band), "hi" = first j with
T < t_min (1 - band); a pixel whose lo and hi differ is a tie.
"""
import numpy as np


def new_state(n):
    """Per-ray compositing state (Sec. 4.1, Eq. 2)."""
    st = {"T": np.ones(n), "C": np.zeros((n, 3)), "n": np.zeros(n, np.int64),
          "levels": np.zeros(n, np.int64)}
    for s in ("lo", "star", "hi"):
        st[s + "_done"] = np.zeros(n, bool)
        st[s + "_C"] = np.zeros((n, 3))
        st[s + "_T"] = np.ones(n)
        st[s + "_n"] = np.zeros(n, np.int64)
    return st


def thresholds(t_min, band):
    """Termination thresholds with the tie band around t_min (reading R15)."""
    return {"lo": t_min * (1.0 + band), "star": t_min, "hi": t_min * (1.0 - band)}


def step(st, rows, sigma, rgb, dt, t_min, band, levels=None):
    """Composite one sample for each ray index in ``rows`` (in order); dt is
    the step length (a scalar, or one per sample).
    Sec. 4.1, Eq. 2; termination per reading R15."""
    alpha = 1.0 - np.exp(-np.asarray(sigma, np.float64) * np.asarray(dt, np.float32).astype(np.float64))
    T = st["T"][rows]
    st["C"][rows] += (T * alpha)[:, None] * rgb
    st["T"][rows] = T * (1.0 - alpha)
    st["n"][rows] += 1
    if levels is not None:
        lv = np.where(st["star_done"][rows], 0, levels)
        st["levels"][rows] += lv
    thr = thresholds(t_min, band)
    for s in ("lo", "star", "hi"):
        hit = (~st[s + "_done"][rows]) & (st["T"][rows] < thr[s])
        if hit.any():
            rr = rows[hit]
            st[s + "_done"][rr] = True
            st[s + "_C"][rr] = st["C"][rr]
            st[s + "_T"][rr] = st["T"][rr]
            st[s + "_n"][rr] = st["n"][rr]


def finish(st):
    """Rays that ran out of samples keep their final state for every end.
    Sec. 4.1, Eq. 2 (final transmittance and alpha)."""
    for s in ("lo", "star", "hi"):
        nd = ~st[s + "_done"]
        st[s + "_C"][nd] = st["C"][nd]
        st[s + "_T"][nd] = st["T"][nd]
        st[s + "_n"][nd] = st["n"][nd]
        st[s + "_done"][:] = True
    return st


def composite_ray(sigma, rgb, dt, t_min, band=1e-4):
    """Single-ray convenience wrapper: returns (C, A, n) at the FP64 rule.
    Sec. 4.1, Eq. 2; reading R15."""
    st = new_state(1)
    rows = np.array([0])
    for j in range(len(sigma)):
        if st["hi_done"][0]:
            break
        step(st, rows, np.array([sigma[j]]), np.asarray(rgb[j], np.float64)[None, :], dt, t_min, band)
    finish(st)
    return st["star_C"][0], 1.0 - st["star_T"][0], int(st["star_n"][0])
