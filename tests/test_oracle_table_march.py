"""Pins for the oracle's lattice range on bounded fields (Sec. 4.3
occupancy grid): with a sample table (Sec. 6 exponential sample distances,
reading R30) and on the uniform lattice (reading R11).

The oracle restricts each ray to a padded range of table indices taken from
an FP64 slab test (``sample_range``).  Nothing about that range is part of
the method: the plain definition visits EVERY table sample k in [0, K) and
keeps the ones whose canonical FP32 cell is inside the grid and occupied.
These tests enumerate that definition here, without the range (own table
recurrence, own canonical position / cell arithmetic, own bit test; for the
uniform lattice every k up to past the farthest reach), and
require the oracle's evaluated lists to equal it exactly on adversarial
rays: from outside the cube, axis-aligned, grazing faces, through corners
and edges, and rays built so that a table sample lands exactly on (or one
FP32 rounding beside) an entry or exit face.  The lists are also checked
against an independent FP64 Amanatides-Woo traversal, and a planted
off-by-one in the range (on the CPU) must be caught.
"""
import math

import numpy as np
import pytest

import oracle.march as om
from oracle.march import dda_traverse, dense_masked_march

F32 = np.float32


def table_field(g, occ, amin, extent, dt, growth, K, cap=100000):
    bits = np.packbits(np.asarray(occ, bool).reshape(-1).astype(np.uint8), bitorder="little")
    bits = np.concatenate([bits, np.zeros((-bits.size) % 4, np.uint8)]).view("<u4")
    return {"occ_res": g, "occ_bits": bits, "aabb_min": np.array(amin, F32), "extent": float(F32(extent)),
            "dt": float(F32(dt)), "max_samples": cap, "step_growth": float(F32(growth)), "max_lattice": K,
            "contraction": 0}


def table_recurrence(dt, growth, K):
    """t_0 = dt/2, t_{k+1} = t_k + max(dt, growth t_k), every op rounded to FP32."""
    dt, growth = F32(dt), F32(growth)
    t = [F32(F32(0.5) * dt)]
    for _ in range(K - 1):
        g = F32(growth * t[-1])
        t.append(F32(t[-1] + (g if g > dt else dt)))
    return np.array(t, F32)


def brute_force_lists(field, occ, o, d):
    """Every table index k in [0, K), in order: kept iff the FP32 canonical
    cell of o + t_k d is inside the G^3 grid and its bit is set (capped)."""
    g = int(field["occ_res"])
    tab = table_recurrence(field["dt"], field["step_growth"], int(field["max_lattice"]))
    amin = np.asarray(field["aabb_min"], F32)
    cs = F32(np.float64(g) / np.float64(F32(field["extent"])))
    out = []
    for r in range(o.shape[0]):
        x = [F32(o[r, a]) + tab * F32(d[r, a]) for a in range(3)]          # FP32: product, then sum
        c = [np.floor(((x[a] - amin[a]).astype(F32) * cs).astype(F32)).astype(np.int64) for a in range(3)]
        inside = (c[0] >= 0) & (c[0] < g) & (c[1] >= 0) & (c[1] < g) & (c[2] >= 0) & (c[2] < g)
        keep = np.zeros(tab.size, bool)
        idx = np.nonzero(inside)[0]
        keep[idx] = occ[c[2][idx], c[1][idx], c[0][idx]]
        ks = np.nonzero(keep)[0][:int(field["max_samples"])]
        out.append(ks.tolist())
    return out


def boundary_rays(g, amin, extent, tab, rng, n=120):
    """Rays on which a table sample lands exactly on, or one FP32 step
    beside, an entry or exit face of the cube."""
    amin = np.asarray(amin, np.float64)
    o, d = [], []
    for _ in range(n):
        a = int(rng.integers(3))
        k = int(rng.integers(1, tab.size - 1))
        s = 1.0 if rng.uniform() < 0.5 else -1.0
        dirv = rng.standard_normal(3) * 0.3
        dirv[a] = s
        dirv /= np.linalg.norm(dirv)
        dirv = dirv.astype(F32)
        face = amin[a] + (0.0 if rng.uniform() < 0.5 else extent)
        # place o so that sample k meets the face on axis a (in FP32), then nudge
        p = amin + extent * rng.uniform(0.1, 0.9, 3)
        p[a] = face
        org = (p - tab[k].astype(np.float64) * dirv.astype(np.float64)).astype(F32)
        nudge = int(rng.integers(-2, 3))
        org[a] = np.nextafter(org[a], F32(np.inf if nudge > 0 else -np.inf)) if nudge else org[a]
        o.append(org)
        d.append(dirv)
    return np.array(o, F32), np.array(d, F32)


def adversarial_rays(g, extent, amin, rng, n_rand=150):
    amin = np.array(amin)
    o, d = [], []
    c = amin + extent * 0.5
    for a in range(3):
        for s in (1, -1):
            e = np.zeros(3)
            e[a] = s
            o += [c, c - 2 * extent * e, amin + extent * np.array([0.25, 0.5, 0.75]), c + 3 * extent * e]
            d += [e, e, e, e]
    cell = extent / g
    for k in range(g + 1):
        o += [amin + np.array([k * cell, 0.37 * extent, -2 * extent])]
        d += [np.array([0.0, 0.0, 1.0])]
        o += [amin + np.array([k * cell, k * cell, -extent])]
        d += [np.array([0.0, 0.0, 1.0])]
    o += [amin - 0.5 * extent * np.ones(3), amin + 1.5 * extent * np.ones(3)]   # diagonals through corners
    d += [np.ones(3), -np.ones(3)]
    o += [amin + np.array([-1e-3, 0.5, 0.5]) * extent]                         # grazing the x = amin face
    d += [np.array([1e-7, 1.0, 0.0])]
    for _ in range(n_rand):
        o.append(amin + extent * rng.uniform(-1.5, 2.5, 3))
        o_to = amin + extent * rng.uniform(0, 1, 3)
        d.append(o_to - o[-1])
    o = np.array(o, F32)
    d = np.array(d, np.float64)
    d = (d / np.linalg.norm(d, axis=1, keepdims=True)).astype(F32)
    return o, d


CASES = [  # (G, growth, K, dt as a fraction of the cell, extent, amin)
    (1, 0.05, 400, 0.31, 1.0, (0.0, 0.0, 0.0)),
    (2, 0.02, 600, 0.17, 1.7, (-0.3, 0.2, 1.0)),
    (3, 0.1, 300, 0.23, 2.5, (1.0, -2.0, 0.5)),
    (4, 0.004, 900, 0.11, 1.0, (-0.5, -0.5, -0.5)),
    (8, 0.03, 700, 0.13, 3.2, (0.0, 0.0, 0.0)),
    (8, 0.25, 60, 0.4, 3.2, (0.0, 0.0, 0.0)),        # a short table that ends inside the cube
]


def _oracle_lists(f, o, d):
    ks, counts = dense_masked_march(f, o, d)
    return [ks[r, :counts[r]].tolist() for r in range(o.shape[0])]


@pytest.mark.parametrize("case", range(len(CASES)))
def test_table_march_equals_unrestricted_enumeration(case):
    g, growth, K, dtf, extent, amin = CASES[case]
    rng = np.random.default_rng(100 + case)
    occ = rng.uniform(size=(g, g, g)) < 0.55
    occ[0, 0, 0] = occ[-1, -1, -1] = occ[0, -1, 0] = True
    f = table_field(g, occ, amin, extent, dtf * extent / g, growth, K)
    tab = table_recurrence(f["dt"], growth, K)
    o1, d1 = adversarial_rays(g, extent, amin, rng)
    o2, d2 = boundary_rays(g, amin, extent, tab, rng)
    o, d = np.concatenate([o1, o2]), np.concatenate([d1, d2])
    want = brute_force_lists(f, occ, o, d)
    got = _oracle_lists(f, o, d)
    bad = [r for r in range(o.shape[0]) if got[r] != want[r]]
    assert not bad, f"{len(bad)} rays differ, e.g. ray {bad[0]}: oracle {got[bad[0]]} brute force {want[bad[0]]}"
    assert sum(len(w) for w in want) > 50


def test_table_march_keeps_face_samples_and_cap():
    # a sample placed exactly on the entry face (cell 0) and on the exit face
    # (outside: cell G) along an axis ray; the cap truncates in k order
    g, extent = 4, 1.0
    occ = np.ones((g, g, g), bool)
    f = table_field(g, occ, (0, 0, 0), extent, 0.05, 0.1, 200)
    tab = table_recurrence(f["dt"], 0.1, 200)
    k_in = 7
    o = np.array([[F32(0.0) - tab[k_in], 0.5, 0.5]], F32)
    d = np.array([[1.0, 0.0, 0.0]], F32)
    want = brute_force_lists(f, occ, o, d)[0]
    assert want and want[0] == k_in, "the face sample is inside the grid by the canonical test"
    assert _oracle_lists(f, o, d)[0] == want
    f5 = dict(f, max_samples=5)
    assert _oracle_lists(f5, o, d)[0] == want[:5]


@pytest.mark.parametrize("case", [1, 4])
def test_table_march_agrees_with_independent_dda(case):
    g, growth, K, dtf, extent, amin = CASES[case]
    rng = np.random.default_rng(200 + case)
    occ = rng.uniform(size=(g, g, g)) < 0.5
    f = table_field(g, occ, amin, extent, dtf * extent / g, growth, K)
    tab = table_recurrence(f["dt"], growth, K).astype(np.float64)
    o, d = adversarial_rays(g, extent, amin, rng, n_rand=100)
    got = _oracle_lists(f, o, d)
    s = g / np.float64(F32(extent))
    checked = 0
    for r in range(o.shape[0]):
        expect = set()
        for (t0, t1, cell) in dda_traverse(o[r], d[r], amin, extent, g):
            if occ[cell[2], cell[1], cell[0]]:
                expect |= set(np.nonzero((tab > t0) & (tab < t1))[0].tolist())
        diff = expect ^ set(got[r])
        # ambiguous: samples within 1e-4 cells of a cell face (FP32 vs FP64 position)
        amb = set()
        for k in diff:
            q = (o[r].astype(np.float64) + tab[k] * d[r].astype(np.float64) - np.asarray(amin)) * s
            fr = q - np.floor(q)
            if np.any(np.minimum(fr, 1 - fr) < 1e-4):
                amb.add(k)
        assert diff <= amb, (r, sorted(diff - amb))
        checked += len(got[r])
    assert checked > 0


def test_planted_range_off_by_one_is_caught(monkeypatch):
    """The pin has teeth: an oracle whose padded range starts one index too
    late, or stops one too early, fails the unrestricted enumeration."""
    g, growth, K, dtf, extent, amin = CASES[3]
    rng = np.random.default_rng(103)
    occ = np.ones((g, g, g), bool)
    f = table_field(g, occ, amin, extent, dtf * extent / g, growth, K)
    tab = table_recurrence(f["dt"], growth, K)
    o, d = boundary_rays(g, amin, extent, tab, rng, n=200)
    want = brute_force_lists(f, occ, o, d)
    original = om.sample_range
    for shift_lo, shift_hi in ((1, 0), (0, -2)):
        def mutated(field, oo, dd, _lo=shift_lo, _hi=shift_hi):
            lo, hi = original(field, oo, dd)
            return lo + _lo, np.where(hi >= 0, hi + _hi, hi)
        monkeypatch.setattr(om, "sample_range", mutated)
        got = _oracle_lists(f, o, d)
        assert any(got[r] != want[r] for r in range(o.shape[0])), (shift_lo, shift_hi)
    monkeypatch.setattr(om, "sample_range", original)
    assert _oracle_lists(f, o, d) == want


def brute_force_uniform(field, occ, o, d, k_max):
    """Every uniform lattice index k in [0, k_max), t_k = (k + 1/2) dt in
    FP32, kept iff its canonical FP32 cell is inside the grid and set."""
    g = int(field["occ_res"])
    k = np.arange(k_max)
    tk = ((k.astype(F32) + F32(0.5)) * F32(field["dt"])).astype(F32)
    amin = np.asarray(field["aabb_min"], F32)
    cs = F32(np.float64(g) / np.float64(F32(field["extent"])))
    out = []
    for r in range(o.shape[0]):
        c = [np.floor(((F32(o[r, a]) + tk * F32(d[r, a])) - amin[a]).astype(F32) * cs).astype(np.int64)
             for a in range(3)]
        inside = (c[0] >= 0) & (c[0] < g) & (c[1] >= 0) & (c[1] < g) & (c[2] >= 0) & (c[2] < g)
        keep = np.zeros(k_max, bool)
        idx = np.nonzero(inside)[0]
        keep[idx] = occ[c[2][idx], c[1][idx], c[0][idx]]
        out.append(np.nonzero(keep)[0][:int(field["max_samples"])].tolist())
    return out


@pytest.mark.parametrize("g", [1, 3, 8])
def test_uniform_march_equals_unrestricted_enumeration(g):
    """The uniform lattice (reading R11): the oracle's padded k range never
    drops a sample the unrestricted enumeration keeps, also for cameras a
    thousand cube edges away whose rays graze the cube (FP32 positions
    there carry errors of a large fraction of a step)."""
    rng = np.random.default_rng(300 + g)
    amin, extent = (0.25, -1.0, 2.0), 1.3
    occ = rng.uniform(size=(g, g, g)) < 0.6
    occ[0, 0, 0] = occ[-1, -1, -1] = True
    dt = extent * math.sqrt(3) / (5 * g)
    f = table_field(g, occ, amin, extent, dt, 0.0, 1)
    del f["step_growth"], f["max_lattice"]
    o1, d1 = adversarial_rays(g, extent, amin, rng, n_rand=120)
    # far cameras aimed at a face, an edge or a corner of the cube (grazing)
    far_o, far_d = [], []
    am = np.asarray(amin, np.float64)
    for i in range(24):
        target = am + extent * np.array([(i >> 0) & 1, (i >> 1) & 1, (i >> 2) & 1], float)
        target += extent * rng.uniform(-0.02, 0.02, 3) * (i % 3 != 0)
        v = rng.standard_normal(3)
        v /= np.linalg.norm(v)
        far_o.append(target - 1000.0 * extent * v)
        far_d.append(v)
    o = np.concatenate([o1, np.array(far_o, F32)])
    d = np.concatenate([d1, np.array(far_d, F32)])
    d = (d / np.linalg.norm(d.astype(np.float64), axis=1, keepdims=True)).astype(F32)
    reach = np.max(np.linalg.norm(o.astype(np.float64) - (am + extent / 2), axis=1)) + 2 * extent
    want = brute_force_uniform(f, occ, o, d, int(reach / dt) + 8)
    got = _oracle_lists(f, o, d)
    bad = [r for r in range(o.shape[0]) if got[r] != want[r]]
    assert not bad, f"{len(bad)} rays differ, e.g. ray {bad[0]}: oracle {got[bad[0]]} brute force {want[bad[0]]}"
    assert sum(len(w) for w in want) > 20
