"""Multiresolution hash encoding with LOD mip-mapping, FP64.

* Hash grid (Sec. 4, after iNGP): L levels, each a table of T entries of
  F = 2 features; level l has integer resolution N_l (lattice of N_l + 1
  points per axis); trilinear interpolation of the 8 corners.
* Coarse levels are stored densely (App. D): a level is dense when
  (N_l + 1)^3 <= T, index = cx + cy (N_l+1) + cz (N_l+1)^2; otherwise the
  spatial hash (cx*pi1 xor cy*pi2 xor cz*pi3) mod 2^32 mod T with the primes
  stored in the field (iNGP's hash; the paper defers to it).
* LOD (Sec. 4.2.1): sample footprint r_hat = t * r; optimal level
  L* = -log_f(2 s r_hat) in the normalised [0,1]^3 coordinates, plus the LOD
  bias (Sec. 4.2.2); per-level weights w_l of Eq. 3; levels with w_l = 0
  are never read (App. D: the finest levels are zeroed rather than fetched).
  Reading: L* is clamped at 0 so level 0 always has weight 1.

Positions: x_n = (x - aabb_min) / extent in FP64 from the canonical FP32
sample x; p = x_n N_l; base corner i0 = min(floor(p), N_l - 1) (so x_n = 1
uses the last cell with fraction 1).
"""
import numpy as np


def level_star(t, r, field):
    """Optimal LOD level L* (Sec. 4.2.1) plus bias (Sec. 4.2.2), clamped >= 0."""
    rhat_n = np.asarray(t, np.float64) * np.asarray(r, np.float64) / np.float64(np.float32(field["extent"]))
    s = np.float64(np.float32(field["base_res"]))
    f = np.float64(np.float32(field["growth"]))
    ls = -np.log(2.0 * s * rhat_n) / np.log(f) + np.float64(np.float32(field["lod_bias"]))
    return np.maximum(ls, 0.0)


def lod_weights(ls, n_levels):
    """Eq. 3: 1 up to floor(L*), L* - floor(L*) up to ceil(L*), 0 above."""
    ls = np.asarray(ls, np.float64)[..., None]
    lv = np.arange(n_levels, dtype=np.float64)
    fl, ce = np.floor(ls), np.ceil(ls)
    return np.where(lv <= fl, 1.0, np.where(lv <= ce, ls - fl, 0.0))


def is_dense(n_l, table_size):
    """Dense storage of a level whose (N+1)^3 lattice points fit the table
    (Sec. 4, after iNGP; reading R7)."""
    return (int(n_l) + 1) ** 3 <= int(table_size)


def level_index(c, n_l, table_size, primes):
    """Table index of integer lattice corners c [..., 3] at one level.
    Dense index or the iNGP spatial hash (Sec. 4; reading R9)."""
    c = np.asarray(c, np.int64)
    if is_dense(n_l, table_size):
        s = int(n_l) + 1
        return c[..., 0] + s * (c[..., 1] + s * c[..., 2])
    cu = c.astype(np.uint64)
    p = [np.uint64(int(v)) for v in primes]
    h = (cu[..., 0] * p[0]) ^ (cu[..., 1] * p[1]) ^ (cu[..., 2] * p[2])
    h &= np.uint64(0xFFFFFFFF)
    return (h % np.uint64(table_size)).astype(np.int64)


def encode(field, x32, weights=None):
    """Features [n, 2L] (level-major, feature fastest) for FP32 positions.

    weights: [n, L] LOD weights or None (all levels weight 1).
    Sec. 4 (multiresolution hash grid), Sec. 4.2.1 Eq. 3 weights, App. D
    (levels of weight 0 are not read); readings R8, R10."""
    x32 = np.asarray(x32, np.float32)
    n = x32.shape[0]
    L = int(field["n_levels"])
    T = 1 << int(field["log2_T"])
    tables = field["tables"]
    amin = np.asarray(field["aabb_min"], np.float32).astype(np.float64)
    extent = np.float64(np.float32(field["extent"]))
    xn = (x32.astype(np.float64) - amin) / extent
    feats = np.zeros((n, 2 * L))
    for l in range(L):
        w = np.ones(n) if weights is None else weights[:, l]
        act = np.nonzero(w > 0)[0]
        if act.size == 0:
            continue
        N = int(field["level_res"][l])
        p = xn[act] * N
        i0 = np.clip(np.floor(p), 0, N - 1)
        fr = p - i0
        i0 = i0.astype(np.int64)
        acc = np.zeros((act.size, 2))
        for corner in range(8):
            dlt = np.array([(corner >> a) & 1 for a in range(3)])
            idx = level_index(i0 + dlt, N, T, field["hash_primes"])
            val = tables[l][idx].astype(np.float64)
            wt = np.prod(np.where(dlt == 1, fr, 1.0 - fr), axis=-1)
            acc += wt[:, None] * val
        feats[act, 2 * l:2 * l + 2] = w[act, None] * acc
    return feats
