"""Pins for the oracle's hash-grid encoding (Sec. 4 after iNGP, App. D dense
coarse levels) against closed forms, invariants and scipy's independent
trilinear interpolator."""
import numpy as np
import pytest
from scipy.interpolate import RegularGridInterpolator

from oracle.encoding import encode, is_dense, level_index

PRIMES = np.array([1, 2654435761, 805459861], np.uint32)


def small_field(res, log2_T, seed=0, amin=(0.0, 0.0, 0.0), extent=1.0, dtype=np.float32):
    rng = np.random.default_rng(seed)
    L = len(res)
    return {"n_levels": L, "log2_T": log2_T, "level_res": np.array(res, np.uint32),
            "hash_primes": PRIMES, "aabb_min": np.array(amin, np.float32), "extent": extent,
            "tables": rng.uniform(-1, 1, size=(L, 1 << log2_T, 2)).astype(dtype)}


def test_dense_index_is_bijection():
    for N, T in ((4, 1 << 7), (16, 1 << 13), (24, 1 << 14)):
        assert is_dense(N, T)
        g = np.stack(np.meshgrid(*[np.arange(N + 1)] * 3, indexing="ij"), -1).reshape(-1, 3)
        idx = level_index(g, N, T, PRIMES)
        assert sorted(idx.tolist()) == list(range((N + 1) ** 3))


def test_hashed_index_in_range_and_prime_structure():
    N, T = 100, 1 << 10
    assert not is_dense(N, T)
    rng = np.random.default_rng(1)
    c = rng.integers(0, N + 1, size=(5000, 3))
    idx = level_index(c, N, T, PRIMES)
    assert idx.min() >= 0 and idx.max() < T
    # pi_1 = 1: along x with y = z = 0 the hash is the coordinate itself (mod T)
    cx = np.stack([np.arange(N + 1), np.zeros(N + 1, int), np.zeros(N + 1, int)], -1)
    assert np.array_equal(level_index(cx, N, T, PRIMES), np.arange(N + 1) % T)
    # (0,1,0) -> pi_2 mod T, (0,0,1) -> pi_3 mod T, xor-combination of the axes
    assert level_index(np.array([[0, 1, 0]]), N, T, PRIMES)[0] == 2654435761 % T
    assert level_index(np.array([[0, 0, 1]]), N, T, PRIMES)[0] == 805459861 % T
    a = level_index(np.array([[3, 5, 7]]), N, T, PRIMES)[0]
    b = (level_index(np.array([[3, 0, 0]]), N, T, PRIMES)[0]
         ^ level_index(np.array([[0, 5, 0]]), N, T, PRIMES)[0]
         ^ level_index(np.array([[0, 0, 7]]), N, T, PRIMES)[0])
    assert a == b


def test_feature_at_lattice_point_equals_table_entry():
    f = small_field([4, 8, 32], 9)
    T = 1 << 9
    for l, N in enumerate([4, 8, 32]):
        c = np.array([[0, 0, 0], [1, 2, 3], [N, N, N], [N - 1, 0, N]])
        x = (c / N).astype(np.float32)
        assert np.all((c / N).astype(np.float32).astype(np.float64) * N == c)  # exact grid points
        w = np.zeros((len(c), 3))
        w[:, l] = 1.0
        feats = encode(f, x, w)
        idx = level_index(c, N, T, PRIMES)
        np.testing.assert_allclose(feats[:, 2 * l:2 * l + 2], f["tables"][l][idx], atol=1e-12)


def test_dense_level_matches_scipy_trilinear():
    N, log2_T = 12, 12
    f = small_field([N], log2_T, seed=3, amin=(-1.0, 0.5, 2.0), extent=2.0)
    grid_vals = np.zeros((N + 1, N + 1, N + 1, 2))
    for cz in range(N + 1):
        for cy in range(N + 1):
            for cx in range(N + 1):
                grid_vals[cx, cy, cz] = f["tables"][0][cx + (N + 1) * (cy + (N + 1) * cz)]
    ax = np.arange(N + 1) / N
    rng = np.random.default_rng(4)
    x = (np.array([-1.0, 0.5, 2.0]) + 2.0 * rng.uniform(0, 1, size=(3000, 3))).astype(np.float32)
    feats = encode(f, x)
    xn = (x.astype(np.float64) - np.array([-1.0, 0.5, 2.0])) / 2.0
    for k in range(2):
        ref = RegularGridInterpolator((ax, ax, ax), grid_vals[..., k], method="linear")(xn)
        np.testing.assert_allclose(feats[:, k], ref, atol=1e-12)


def test_constant_table_gives_constant_feature_and_weights_scale():
    f = small_field([5, 40, 77], 8)
    f["tables"][:] = np.array([0.25, -0.5], np.float32)
    x = np.random.default_rng(5).uniform(0, 1, size=(500, 3)).astype(np.float32)
    feats = encode(f, x)
    np.testing.assert_allclose(feats, np.tile([0.25, -0.5], 3)[None].repeat(500, 0), atol=1e-12)
    w = np.tile([1.0, 0.3, 0.0], (500, 1))
    fw = encode(f, x, w)
    np.testing.assert_allclose(fw[:, 2:4], 0.3 * feats[:, 2:4], atol=1e-12)
    assert np.all(fw[:, 4:6] == 0)


def test_linear_along_cell_edge_and_upper_boundary():
    N = 7
    f = small_field([N], 12, seed=6)
    y0, z0 = 2 / N, 5 / N
    ts = np.linspace(0, 1, 11)
    x = np.stack([(3 + ts) / N, np.full_like(ts, y0), np.full_like(ts, z0)], -1).astype(np.float32)
    xn = x.astype(np.float64)
    feats = encode(f, x)
    idx = level_index(np.array([[3, 2, 5], [4, 2, 5]]), N, 1 << 12, PRIMES)
    a, b = f["tables"][0][idx[0]], f["tables"][0][idx[1]]
    fr = xn[:, 0] * N - 3
    ok = (fr >= 0) & (fr < 1)
    ref = (1 - fr)[:, None] * a + fr[:, None] * b
    np.testing.assert_allclose(feats[ok], ref[ok], atol=1e-6)
    # x_n = 1 exactly: the far lattice corner's value (clamped base cell, fraction 1)
    top = encode(f, np.ones((1, 3), np.float32))
    idx_top = level_index(np.array([[N, N, N]]), N, 1 << 12, PRIMES)
    np.testing.assert_allclose(top[0], f["tables"][0][idx_top[0]], atol=1e-12)
