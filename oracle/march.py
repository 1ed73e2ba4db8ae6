"""Occupancy-grid lattice march -- Sec. 4.3 (binary occupancy grid used to
skip free space and cut hash queries and MLP evaluations).

Plain definition (the result occupancy skipping must reach exactly): visit
EVERY lattice sample t_k = (k + 1/2) dt of the ray, keep the ones whose cell
in the G^3 bitfield is set.  Readings taken here (the paper trains with
exponential spacing and gives no render-time sampler):

* uniform lattice from the ray origin, t_k = (k + 0.5) dt, delta = dt;
* the sample position and its cell are computed on the canonical FP32 ray,
  each op rounded:  t_k = (k + 0.5) * dt,  x = o + t_k * d,
  q = (x - aabb_min) * cell_scale with cell_scale = fp32(G / extent),
  cell = floor(q); the sample is valid iff 0 <= cell < G on every axis;
* the k range comes from an FP64 slab test of the cube grown by a bound on
  the FP32 position error, padded by one step on each side, so membership is
  decided by the canonical test alone;
* "max samples per ray" caps EVALUATED samples (valid and occupied).

``dda_traverse`` is an independent FP64 Amanatides-Woo voxel traversal used
only to pin the march: its cell intervals must contain the same samples.
"""
import numpy as np

from .geometry import contract32, is_contracted, lattice_table, pipeline_field

F32 = np.float32


def cell_scale(field):
    """Cells per unit length of the occupancy grid (Sec. 4.3; reading R13)."""
    return F32(np.float64(field["occ_res"]) / np.float64(F32(field["extent"])))


# Bound on how far a canonical FP32 sample position (and its cell
# coordinate) can stray from the exact point o + t d: every op of reading
# R13 rounds once (relative 2^-24), so the error stays below
# 2^-22 (|o| + t + |aabb_min| + 2 extent) in world units; the range below uses
# four times that (ERR_REL = 2^-20).
ERR_REL = 2.0 ** -20


def reach_interval(o, d, aabb_min, extent):
    """[t_lo, t_hi] (FP64) outside of which no canonical FP32 sample of the
    rays o + t d can pass the cell test of the cube [amin, amin + extent]:
    the slab test of a box that grows with t by the FP32 position error
    bound, c0 + c1 t per side.  t_hi < t_lo when no sample can.
    Sec. 4.3; reading R13 (membership is decided by the canonical test alone,
    so the range only has to contain every sample that test could keep)."""
    o64 = np.asarray(o, np.float64)
    d64 = np.asarray(d, np.float64)
    lo = np.asarray(aabb_min, F32).astype(np.float64)
    ext = np.float64(F32(extent))
    hi = lo + ext
    c0 = ERR_REL * (np.max(np.abs(o64), axis=-1) + np.max(np.abs(lo)) + 2.0 * ext)
    c1 = ERR_REL
    t_lo = np.zeros(o64.shape[:-1])
    t_hi = np.full(o64.shape[:-1], np.inf)

    def constrain(alpha, beta, ge):
        # t * alpha >= beta (ge) or t * alpha <= beta
        nonlocal t_lo, t_hi
        with np.errstate(divide="ignore", invalid="ignore"):
            r = beta / alpha
        up = (alpha < 0) if ge else (alpha > 0)        # an upper bound on t
        dn = (alpha > 0) if ge else (alpha < 0)        # a lower bound on t
        t_hi = np.where(up, np.minimum(t_hi, r), t_hi)
        t_lo = np.where(dn, np.maximum(t_lo, r), t_lo)
        never = (alpha == 0) & ((beta > 0) if ge else (beta < 0))
        t_hi = np.where(never, -np.inf, t_hi)

    for a in range(3):
        constrain(d64[..., a] + c1, lo[a] - c0 - o64[..., a], True)
        constrain(d64[..., a] - c1, hi[a] + c0 - o64[..., a], False)
    return t_lo, t_hi


def lattice_range(t_lo, t_hi, dt):
    """Inclusive k range [k_lo, k_hi] of lattice samples t_k = (k + 1/2) dt
    that can fall in [t_lo, t_hi], padded by one step (t_k carries its own
    rounding); k_hi = -1 if none.  Sec. 4.3; readings R11 and R13."""
    dt = np.float64(F32(dt))
    hit = t_hi >= t_lo
    with np.errstate(invalid="ignore"):
        lo = np.floor(np.where(hit, t_lo, 0.0) / dt - 0.5) - 1
        hi = np.ceil(np.where(hit, t_hi, 0.0) / dt - 0.5) + 1
    k_lo = np.maximum(lo, 0.0)
    k_hi = np.where(hit, hi, -1.0)
    return k_lo.astype(np.int64), k_hi.astype(np.int64)


def lattice_t(k, dt):
    """Canonical FP32 lattice parameter t_k = (k + 0.5) * dt.  Reading R11 (uniform lattice)."""
    return (np.asarray(k).astype(F32) + F32(0.5)) * F32(dt)


def canonical_positions(o, d, k, dt):
    """FP32 sample positions o + t_k d for o, d [n, 3] and k [n, K].
    Reading R13 (canonical FP32 geometry)."""
    tk = lattice_t(k, dt)
    o = np.asarray(o, F32)
    d = np.asarray(d, F32)
    return np.stack([o[:, a:a + 1] + tk * d[:, a:a + 1] for a in range(3)], axis=-1), tk


def canonical_cells(x, field):
    """Continuous cell coordinates q, integer cells and validity for FP32 x.  Sec. 4.3; reading R13."""
    amin = np.asarray(field["aabb_min"], F32)
    cs = cell_scale(field)
    q = np.stack([(x[..., a] - amin[a]) * cs for a in range(3)], axis=-1)
    c = np.floor(q).astype(np.int64)
    g = int(field["occ_res"])
    valid = np.all((c >= 0) & (c < g), axis=-1)
    return q, c, valid


def occupied(c, valid, field):
    """Occupancy bit of a valid cell (Sec. 4.3)."""
    g = int(field["occ_res"])
    bits = np.asarray(field["occ_bits"], np.uint32)
    cc = np.where(valid[..., None], c, 0)
    idx = cc[..., 0] + g * (cc[..., 1] + g * cc[..., 2])
    word = bits[idx >> 5]
    return valid & (((word >> (idx & 31).astype(np.uint32)) & 1) == 1)


def uses_table(field):
    """Whether samples come from the FP32 table (Sec. 6; reading R30) rather than the uniform lattice."""
    return is_contracted(field) or float(field.get("step_growth", 0.0)) > 0.0


def sample_points(field, o, d, k):
    """Canonical FP32 sample points for o, d [n, 3] and lattice indices k
    [n, K]: returns (y, t) with y in the coordinates the occupancy and hash
    grids use (world for bounded fields, contracted for unbounded ones).
    Readings R11, R13, R30, R31."""
    if not uses_table(field):
        return canonical_positions(o, d, k, field["dt"])
    tab, _ = lattice_table(field)
    tk = tab[np.clip(k, 0, tab.size - 1)]
    o = np.asarray(o, F32)
    d = np.asarray(d, F32)
    x = np.stack([o[:, a:a + 1] + tk * d[:, a:a + 1] for a in range(3)], axis=-1)
    return (contract32(x, field) if is_contracted(field) else x), tk


def sample_range(field, o, d):
    """Inclusive lattice index range [k_lo, k_hi] worth testing per ray.  Sec. 4.3; readings R11-R14."""
    if is_contracted(field):
        n = o.shape[0]
        return np.zeros(n, np.int64), np.full(n, int(field["max_lattice"]) - 1, np.int64)
    t_lo, t_hi = reach_interval(o, d, field["aabb_min"], field["extent"])
    if not uses_table(field):
        return lattice_range(t_lo, t_hi, field["dt"])
    # table samples: every index whose FP32 entry lies in [t_lo, t_hi], one more on each side
    tab, _ = lattice_table(field)
    hit = t_hi >= t_lo
    lo = np.maximum(np.searchsorted(tab, np.where(hit, t_lo, 0.0), side="left") - 1, 0)
    hi = np.minimum(np.searchsorted(tab, np.where(hit, t_hi, 0.0), side="right"), tab.size - 1)
    return lo.astype(np.int64), np.where(hit & (lo <= hi), hi, -1).astype(np.int64)


def dense_masked_march(field, o, d, chunk=512):
    """Evaluated lattice indices per ray, in increasing k, capped.

    Returns (ks [n, M] int64 padded with -1, counts [n]).
    Sec. 4.3 (occupancy grid), as its plain definition: every lattice sample
    tested; reading R14 for the cap."""
    o = np.asarray(o, F32)
    d = np.asarray(d, F32)
    n = o.shape[0]
    k_lo, k_hi = sample_range(field, o, d)
    pf = pipeline_field(field)
    cap = int(field["max_samples"])
    span = int(np.max(k_hi - k_lo + 1, initial=0))
    rows, cols = [], []
    counts = np.zeros(n, np.int64)
    for c0 in range(0, max(span, 0), chunk):
        off = np.arange(c0, min(c0 + chunk, span))
        k = k_lo[:, None] + off[None, :]
        inr = (k <= k_hi[:, None]) & (counts[:, None] < cap)
        if not inr.any():
            break
        y, _ = sample_points(field, o, d, k)
        _, c, valid = canonical_cells(y, pf)
        ev = occupied(c, valid & inr, pf)
        # cap: keep at most cap - counts samples per ray from this chunk
        rank = np.cumsum(ev, axis=1) + counts[:, None]
        ev &= rank <= cap
        r, cidx = np.nonzero(ev)
        rows.append(r)
        cols.append(k[r, cidx])
        counts += ev.sum(axis=1)
    m = int(counts.max(initial=0))
    ks = np.full((n, max(m, 1)), -1, np.int64)
    if rows:
        r = np.concatenate(rows)
        kk = np.concatenate(cols)
        order = np.lexsort((kk, r))
        r, kk = r[order], kk[order]
        start = np.searchsorted(r, np.arange(n))
        pos = np.arange(r.size) - start[r]
        ks[r, pos] = kk
    return ks, counts


def dda_traverse(o, d, aabb_min, extent, g):
    """Independent FP64 Amanatides-Woo traversal of one ray through the G^3
    grid: list of (t_in, t_out, (cx, cy, cz)) in order of t.  A pin for the
    march of Sec. 4.3, from the published traversal, not from this module."""
    o = np.asarray(o, np.float64)
    d = np.asarray(d, np.float64)
    s = g / np.float64(F32(extent))
    q0 = (o - np.asarray(aabb_min, F32).astype(np.float64)) * s
    dq = d * s
    t_in, t_out = -np.inf, np.inf
    for a in range(3):
        if dq[a] == 0.0:
            if not (0.0 <= q0[a] <= g):
                return []
            continue
        t1, t2 = (0.0 - q0[a]) / dq[a], (g - q0[a]) / dq[a]
        t_in, t_out = max(t_in, min(t1, t2)), min(t_out, max(t1, t2))
    t = max(t_in, 0.0)
    if t_out <= t:
        return []
    p0 = q0 + t * dq
    cell = np.floor(p0)
    # a point exactly on a face belongs to the cell the ray moves into
    cell = np.where((p0 == cell) & (dq < 0), cell - 1, cell)
    cell = np.clip(cell, 0, g - 1).astype(np.int64)
    step = np.sign(dq).astype(np.int64)
    t_max = np.full(3, np.inf)
    t_delta = np.full(3, np.inf)
    for a in range(3):
        if dq[a] != 0.0:
            nxt = cell[a] + (1 if dq[a] > 0 else 0)
            t_max[a] = (nxt - q0[a]) / dq[a]
            t_delta[a] = 1.0 / abs(dq[a])
    out = []
    while True:
        a = int(np.argmin(t_max))
        t_next = min(t_max[a], t_out)
        out.append((t, t_next, tuple(int(v) for v in cell)))
        if t_max[a] >= t_out:
            break
        t = t_max[a]
        cell[a] += step[a]
        t_max[a] += t_delta[a]
        if not (0 <= cell[a] < g):
            break
    return out
