"""Pins for the oracle's occupancy march (Sec. 4.3) and compositing:
brute-force agreement of the dense-masked march with an independent FP64
Amanatides-Woo traversal on tiny and adversarial grids, closed forms of
compositing (constant density, occupied slab), invariants, and whole-render
special cases."""
import math

import numpy as np
import pytest

from oracle import composite as comp
from oracle.march import (canonical_cells, canonical_positions, cell_scale, dda_traverse,
                          dense_masked_march, lattice_t)
from oracle.render import render_fp64

F32 = np.float32


def grid_field(g, occ, amin=(0.0, 0.0, 0.0), extent=1.0, dt=None, cap=100000):
    bits = np.packbits(np.asarray(occ, bool).reshape(-1).astype(np.uint8), bitorder="little")
    pad = (-bits.size) % 4
    bits = np.concatenate([bits, np.zeros(pad, np.uint8)]).view("<u4")
    return {"occ_res": g, "occ_bits": bits, "aabb_min": np.array(amin, F32),
            "extent": float(F32(extent)), "dt": float(F32(dt if dt else extent * math.sqrt(3) / (7 * g))),
            "max_samples": cap}


def adversarial_rays(g, extent, amin, rng, n_rand=200):
    amin = np.array(amin)
    o, d = [], []
    c = amin + extent * 0.5
    for a in range(3):                      # axis-aligned, both senses, from inside and outside
        for s in (1, -1):
            e = np.zeros(3); e[a] = s
            o += [c, c - 2 * extent * e, amin + extent * np.array([0.25, 0.5, 0.75])]
            d += [e, e, e]
    cell = extent / g
    for k in range(g + 1):                  # along cell faces, edges and through corners
        p = amin + np.array([k * cell, 0.37 * extent, 0.61 * extent])
        o += [p - 3 * extent * np.array([0, 1, 0])]
        d += [np.array([0.0, 1.0, 0.0])]
        q = amin + np.array([k * cell, k * cell, -extent])
        o += [q]
        d += [np.array([0.0, 0.0, 1.0])]
    o += [amin - 0.5 * extent * np.ones(3)]  # main diagonal through every corner
    d += [np.ones(3) / math.sqrt(3)]
    o += [amin + np.array([-1e-3, 0.5, 0.5]) * extent]   # grazing the x = amin face
    d += [np.array([1e-7, 1.0, 0.0])]
    for _ in range(n_rand):
        p = amin + extent * rng.uniform(-0.5, 1.5, 3)
        v = rng.standard_normal(3)
        o.append(p)
        d.append(v / np.linalg.norm(v))
    o = np.array(o, F32)
    d = np.array(d)
    d = (d / np.linalg.norm(d, axis=1, keepdims=True)).astype(F32)
    return o, d


@pytest.mark.parametrize("g", [1, 2, 3, 4, 8])
def test_dense_march_equals_independent_dda(g):
    rng = np.random.default_rng(g)
    amin, extent = (-0.3, 0.2, 1.0), 1.7
    occ = rng.uniform(size=(g, g, g)) < 0.5
    occ[0, 0, 0] = occ[-1, -1, -1] = True
    f = grid_field(g, occ, amin, extent)
    o, d = adversarial_rays(g, extent, amin, rng)
    ks, counts = dense_masked_march(f, o, d)
    dt = np.float64(F32(f["dt"]))
    s = g / np.float64(F32(extent))
    checked = 0
    for r in range(o.shape[0]):
        iv = dda_traverse(o[r], d[r], amin, extent, g)
        # every lattice sample whose exact position is strictly inside a DDA
        # interval (margin above FP32 rounding) must be evaluated iff that cell is set
        expect = []
        for (t0, t1, cell) in iv:
            if not occ[cell[2], cell[1], cell[0]]:
                continue
            k0 = max(0, int(math.floor(t0 / dt - 0.5)) - 1)
            k1 = int(math.ceil(t1 / dt - 0.5)) + 1
            for k in range(k0, k1 + 1):
                tau = (k + 0.5) * dt
                if t0 < tau < t1:
                    expect.append(k)
        got = set(ks[r, :counts[r]].tolist())
        # ambiguous samples: within 1e-4 cells of any cell face
        amb = set()
        for k in set(expect) ^ got:
            x, _ = canonical_positions(o[r:r + 1], d[r:r + 1], np.array([[k]]), f["dt"])
            q, _, _ = canonical_cells(x, f)
            frac = q[0, 0] - np.floor(q[0, 0])
            if np.any(np.minimum(frac, 1 - frac) < 1e-4):
                amb.add(k)
        assert (set(expect) - amb) == (got - amb), (r, sorted(set(expect) ^ got))
        checked += len(got)
    assert checked > 0


def test_march_empty_full_and_cap():
    g = 4
    o = np.array([[0.5, 0.5, -0.2], [0.1, 0.9, 0.5]], F32)
    d = np.array([[0, 0, 1], [0.6, -0.8, 0]], F32)
    f0 = grid_field(g, np.zeros((g, g, g)))
    ks, counts = dense_masked_march(f0, o, d)
    assert counts.tolist() == [0, 0]
    f1 = grid_field(g, np.ones((g, g, g)))
    ks, counts = dense_masked_march(f1, o, d)
    # every lattice sample inside the cube is evaluated
    dt = np.float64(F32(f1["dt"]))
    t_in, t_out = 0.2, 1.2
    ref = sum(1 for k in range(1000) if t_in < (k + 0.5) * dt < t_out)
    assert counts[0] == ref
    assert np.all(np.diff(ks[0, :counts[0]]) == 1)
    f2 = grid_field(g, np.ones((g, g, g)), cap=5)
    _, counts2 = dense_masked_march(f2, o, d)
    assert counts2.tolist() == [5, 5]


def test_composite_constant_density_closed_form():
    dt, sigma, c = 0.01, 7.0, np.array([0.2, 0.5, 0.9])
    for n in (1, 5, 40):
        C, A, cnt = comp.composite_ray([sigma] * n, [c] * n, dt, t_min=0.0)
        assert A == pytest.approx(1 - math.exp(-sigma * n * np.float64(F32(dt))), rel=1e-12)
        np.testing.assert_allclose(C, c * A, rtol=1e-12)
        assert cnt == n


def test_composite_invariants_and_termination():
    rng = np.random.default_rng(0)
    for _ in range(50):
        n = rng.integers(1, 60)
        s = rng.exponential(50, n)
        col = rng.uniform(0, 1, (n, 3))
        st = comp.new_state(1)
        Ts = [1.0]
        for j in range(n):
            comp.step(st, np.array([0]), s[j:j + 1], col[j:j + 1], 0.02, 1e-4, 1e-4)
            Ts.append(st["T"][0])
        comp.finish(st)
        Ts = np.array(Ts)
        assert np.all(np.diff(Ts) <= 0) and np.all((Ts >= 0) & (Ts <= 1))
        assert np.all((st["C"] >= 0) & (st["C"] <= 1 - st["T"][0] + 1e-15))
        # stop index is the first sample that brings T below t_min
        below = np.nonzero(Ts[1:] < 1e-4)[0]
        assert st["star_n"][0] == (below[0] + 1 if below.size else n)
        assert st["lo_n"][0] <= st["star_n"][0] <= st["hi_n"][0]
        # error of stopping early is bounded by t_min
        assert np.max(np.abs(st["C"][0] - st["star_C"][0])) <= 1e-4 + 1e-15


def _axis_camera(pos, W=8):
    # forward = +x, right = -y, down = -z (a valid OpenCV c2w)
    R = np.array([[0, 0, 1], [-1, 0, 0], [0, -1, 0]], float)
    fx = 1e6  # nearly parallel rays along +x
    return {"c2w": np.concatenate([R, np.array(pos)[:, None]], 1).astype(F32), "fx": F32(fx),
            "fy": F32(fx), "cx": F32(W / 2), "cy": F32(W / 2)}


def _zero_mlp(b_sigma=0.0, L=2, bands=2):
    return {"W1": np.zeros((2 * L, 64), F32), "b1": np.zeros(64, F32),
            "W2": np.zeros((64, 16), F32), "b2": np.array([b_sigma] + [0] * 15, F32),
            "W3": np.zeros((15 + bands * bands, 64), F32), "b3": np.zeros(64, F32),
            "W4": np.zeros((64, 64), F32), "b4": np.zeros(64, F32),
            "W5": np.zeros((64, 3), F32), "b5": np.zeros(3, F32)}


def _render_field(occ, g=16, b_sigma=0.0, t_min=1e-4):
    f = grid_field(g, occ, (0, 0, 0), 1.0, dt=math.sqrt(3) / 64, cap=64)
    rng = np.random.default_rng(0)
    f.update({"n_levels": 2, "log2_T": 10, "level_res": np.array([4, 40], np.uint32),
              "hash_primes": np.array([1, 2654435761, 805459861], np.uint32),
              "tables": rng.uniform(-0.1, 0.1, (2, 1024, 2)).astype(F32),
              "base_res": 4.0, "growth": 10.0, "mlp": _zero_mlp(b_sigma), "sh_bands": 2,
              "t_min": t_min, "lod_enable": 0, "lod_bias": 0.0, "lod_radius_scale": 1.0})
    return f


def test_render_all_zero_mlp_full_grid_closed_form():
    # zero weights and biases: sigma = e^0 = 1, c = sigmoid(0) = 1/2
    g = 16
    f = _render_field(np.ones((g, g, g)), g)
    cam = _axis_camera([0.5, 0.5, 0.5])
    out = render_fp64(f, [cam], 8, 8)
    dt = np.float64(F32(f["dt"]))
    n = sum(1 for k in range(200) if (k + 0.5) * dt < 0.5 - 1e-6)
    assert np.all(out["n"] == n)
    A = 1 - math.exp(-n * dt)
    np.testing.assert_allclose(out["rgba"][:, 3], A, rtol=1e-12)
    np.testing.assert_allclose(out["rgba"][:, :3], 0.5 * A, rtol=1e-12)


def test_render_occupied_slab_opacity():
    # a slab of occupied cells x in [6/16, 10/16): opacity 1 - exp(-sigma L), L = n dt
    g = 16
    occ = np.zeros((g, g, g), bool)
    occ[:, :, 6:10] = True
    sigma = 3.0
    f = _render_field(occ, g, b_sigma=math.log(sigma))
    sigma = math.exp(float(F32(math.log(sigma))))   # the bias is stored in FP32
    cam = _axis_camera([0.05, 0.5, 0.5])
    out = render_fp64(f, [cam], 8, 8)
    dt = np.float64(F32(f["dt"]))
    n = sum(1 for k in range(200) if 6 / 16 < 0.05 + (k + 0.5) * dt < 10 / 16)
    assert np.all(out["n"] == n)
    np.testing.assert_allclose(out["rgba"][:, 3], 1 - np.exp(-sigma * n * dt), rtol=1e-9)
    np.testing.assert_allclose(out["rgba"][:, 0], 0.5 * (1 - np.exp(-sigma * n * dt)), rtol=1e-9)


def test_render_empty_grid_is_black_and_termination_tie_bookkeeping():
    g = 16
    f = _render_field(np.zeros((g, g, g)), g)
    out = render_fp64(f, [_axis_camera([0.5, 0.5, 0.5])], 8, 8)
    assert np.all(out["rgba"] == 0) and np.all(out["n"] == 0) and not out["tie"].any()
    # dense opaque grid: termination happens and is counted
    f = _render_field(np.ones((g, g, g)), g, b_sigma=math.log(80.0))
    out = render_fp64(f, [_axis_camera([0.2, 0.5, 0.5])], 8, 8)
    dt = np.float64(F32(f["dt"]))
    s80 = math.exp(float(F32(math.log(80.0))))
    T, k = 1.0, 0
    while T >= 1e-4:
        T *= math.exp(-s80 * dt)
        k += 1
    assert np.all(out["n"] == k)
    assert np.all(out["rgba"][:, 3] > 1 - 1e-4)
