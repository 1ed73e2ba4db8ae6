"""Seeded synthetic fields and camera paths.

This module only *draws inputs*: hash tables, MLP weights, occupancy
bitfields and camera poses with the shapes of the paper's workloads
(room-scale scenes, 16 levels of 2 features, 64-wide MLPs, Sec. 6
"Results"; stereo 2K x 2K eye buffers, Sec. 6.2).  It contains none of the
renderer's arithmetic (no ray marching, encoding, MLP evaluation or
compositing), so both the HIP renderer and the CPU oracle can consume what
it produces without sharing any method code.

RNG: ``numpy.random.default_rng(1000 * block + part)``, one seed block per
workload (1 blob field, 2 room, 4 house, 5 serving room) and part 1 = tables,
2 = MLP weights, 3 = occupancy, 4 = cameras.

A *field* is a plain dict of numpy arrays and scalars:

  n_levels, log2_T, n_feat (=2), level_res[L] (uint32), hash_primes[3],
  base_res (s), growth (f), tables [L][T][2] (float32 or float16),
  mlp: dict W1,b1,W2,b2,W3,b3,W4,b4,W5,b5 (float32, W row-major [in][out]),
  sh_bands, occ_res (G), occ_bits (uint32 words, bit i = x + G*(y + G*z),
  LSB first), aabb_min[3], extent, dt, max_samples, t_min,
  lod_enable, lod_bias, lod_radius_scale.

A *camera* is a dict: c2w (float32 3x4, OpenCV axes: +x right, +y down,
+z forward), fx, fy, cx, cy (float32 scalars).
"""
from __future__ import annotations

import json
import math
import os

import numpy as np

HASH_PRIMES = (1, 2654435761, 805459861)
MLP_HIDDEN = 64
GEO_OUT = 16


def rng_for(block: int, part: int) -> np.random.Generator:
    return np.random.default_rng(1000 * block + part)


# ----------------------------------------------------------------------------
# field pieces
# ----------------------------------------------------------------------------

def level_resolutions(n_levels: int, base: float, growth: float) -> np.ndarray:
    """Integer lattice resolution per level, floor(s * f^l) (iNGP convention).

    A tiny epsilon keeps e.g. 16 * (256^(1/15))^15 at 4096 instead of 4095."""
    return np.array([math.floor(base * growth ** l + 1e-6) for l in range(n_levels)],
                    dtype=np.uint32)


def glorot(rng, fan_in, fan_out):
    lim = math.sqrt(6.0 / (fan_in + fan_out))
    return rng.uniform(-lim, lim, size=(fan_in, fan_out)).astype(np.float32)


def density_bias(t_min: float, n_hit: float, dt: float) -> float:
    """Output bias of the density head chosen so that a ray crossing ``n_hit``
    occupied lattice samples reaches transmittance t_min (a trained scene's
    surfaces are opaque within a few samples)."""
    return math.log(math.log(1.0 / t_min) / (n_hit * dt))


def make_mlp(rng, n_levels: int, sh_bands: int, b_sigma: float) -> dict:
    d_in = 2 * n_levels
    c_in = (GEO_OUT - 1) + sh_bands * sh_bands
    m = {
        "W1": glorot(rng, d_in, MLP_HIDDEN), "b1": np.zeros(MLP_HIDDEN, np.float32),
        "W2": glorot(rng, MLP_HIDDEN, GEO_OUT), "b2": np.zeros(GEO_OUT, np.float32),
        "W3": glorot(rng, c_in, MLP_HIDDEN), "b3": np.zeros(MLP_HIDDEN, np.float32),
        "W4": glorot(rng, MLP_HIDDEN, MLP_HIDDEN), "b4": np.zeros(MLP_HIDDEN, np.float32),
        "W5": glorot(rng, MLP_HIDDEN, 3), "b5": np.zeros(3, np.float32),
    }
    m["b2"][0] = np.float32(b_sigma)
    return m


def pack_bits(occ_zyx: np.ndarray) -> np.ndarray:
    """Pack a boolean [z][y][x] grid into LSB-first uint32 words."""
    g = occ_zyx.shape[0]
    flat = np.ascontiguousarray(occ_zyx, dtype=bool).reshape(-1)
    pad = (-flat.size) % 32
    if pad:
        flat = np.concatenate([flat, np.zeros(pad, bool)])
    b = np.packbits(flat.astype(np.uint8), bitorder="little")
    return b.view("<u4").astype(np.uint32, copy=False).copy()


def unpack_bits(words: np.ndarray, g: int) -> np.ndarray:
    b = np.unpackbits(np.asarray(words, "<u4").view(np.uint8), bitorder="little")
    return b[: g * g * g].astype(bool).reshape(g, g, g)


def blob_occupancy(rng, g: int, n_blobs: int = 8, frac: float = 0.10) -> np.ndarray:
    centres = rng.uniform(0.15, 0.85, size=(n_blobs, 3))
    stds = rng.uniform(0.04, 0.10, size=n_blobs)
    c = (np.arange(g) + 0.5) / g
    z, y, x = np.meshgrid(c, c, c, indexing="ij")
    score = np.zeros((g, g, g))
    for (cx, cy, cz), s in zip(centres, stds):
        score += np.exp(-((x - cx) ** 2 + (y - cy) ** 2 + (z - cz) ** 2) / (2 * s * s))
    thr = np.quantile(score, 1.0 - frac)
    return score > thr


def room_occupancy(rng, g: int, frac: float = 0.05) -> np.ndarray:
    """Unit-cube room: 1-cell shell plus furniture box shells and shelves."""
    occ = np.zeros((g, g, g), bool)
    occ[0], occ[-1] = True, True
    occ[:, 0], occ[:, -1] = True, True
    occ[:, :, 0], occ[:, :, -1] = True, True
    lo, hi = int(0.05 * g), int(0.40 * g)
    while occ.mean() < frac:
        if rng.uniform() < 0.75:     # furniture: hollow box shell standing on the floor
            sx, sy = rng.integers(g // 20, g // 4, size=2)
            sz = rng.integers(g // 25, int(0.24 * g))
            x0 = rng.integers(1, g - 1 - sx)
            y0 = rng.integers(1, g - 1 - sy)
            z0, z1 = 1, 1 + sz
            x1, y1 = x0 + sx, y0 + sy
            occ[z0:z1, y0:y1, x0] = occ[z0:z1, y0:y1, x1 - 1] = True
            occ[z0:z1, y0, x0:x1] = occ[z0:z1, y1 - 1, x0:x1] = True
            occ[z1 - 1, y0:y1, x0:x1] = True
        else:                        # shelf plane on a wall, away from eye height
            depth = rng.integers(g // 16, g // 6)
            length = rng.integers(g // 6, g // 2)
            z = rng.integers(lo, hi) if rng.uniform() < 0.5 else rng.integers(int(0.6 * g), g - 2)
            a0 = rng.integers(1, g - 1 - length)
            wall = rng.integers(4)
            if wall == 0:
                occ[z, a0:a0 + length, 1:1 + depth] = True
            elif wall == 1:
                occ[z, a0:a0 + length, g - 1 - depth:g - 1] = True
            elif wall == 2:
                occ[z, 1:1 + depth, a0:a0 + length] = True
            else:
                occ[z, g - 1 - depth:g - 1, a0:a0 + length] = True
    return occ


def make_tables(rng, n_levels, log2_T, dist: str, dtype=np.float32) -> np.ndarray:
    shape = (n_levels, 1 << log2_T, 2)
    if dist == "uniform":
        t = rng.uniform(-0.1, 0.1, size=shape).astype(np.float32)
    else:  # N(0, variance 1e-2)
        t = rng.standard_normal(size=shape, dtype=np.float32) * np.float32(0.1)
    return t.astype(dtype)


def _field(**kw) -> dict:
    f = dict(n_feat=2, hash_primes=np.array(HASH_PRIMES, np.uint32), lod_bias=0.0,
             lod_radius_scale=1.0)
    f.update(kw)
    f["aabb_min"] = np.asarray(f["aabb_min"], np.float32)
    f["extent"] = float(np.float32(f["extent"]))
    f["dt"] = float(np.float32(f["dt"]))
    f["t_min"] = float(np.float32(f["t_min"]))
    f["base_res"] = float(np.float32(f["base_res"]))
    f["growth"] = float(np.float32(f["growth"]))
    return f


# ----------------------------------------------------------------------------
# the five workloads
# ----------------------------------------------------------------------------

def field_blobs64(extent: float = 1.0, table_dtype=np.float32) -> dict:
    """64^2 / 8 levels / T=2^14 / 64^3 blob bitfield (~10 %), unit cube."""
    L, log2_T, s, f = 8, 14, 16.0, 1.5
    dt = np.float32(extent * math.sqrt(3.0) / 64.0)
    g = 64
    occ = blob_occupancy(rng_for(1, 3), g, 8, 0.10)
    return _field(
        name="blobs64", n_levels=L, log2_T=log2_T, level_res=level_resolutions(L, s, f),
        base_res=s, growth=f, tables=make_tables(rng_for(1, 1), L, log2_T, "uniform", table_dtype),
        mlp=make_mlp(rng_for(1, 2), L, 2, density_bias(1e-4, 4.0, float(dt))), sh_bands=2,
        occ_res=g, occ_bits=pack_bits(occ), aabb_min=[0.0, 0.0, 0.0], extent=extent,
        dt=dt, max_samples=64, t_min=1e-4, lod_enable=0)


def field_room256(log2_T: int = 19, table_dtype=np.float32, seed_block: int = 2) -> dict:
    """1024^2 / 16 levels / T=2^19 / 256^3 room bitfield (~5 %), LOD on."""
    L, s, nmax = 16, 16.0, 4096.0
    f64 = (nmax / s) ** (1.0 / (L - 1))
    f = float(np.float32(f64))
    g = 256
    dt = np.float32(math.sqrt(3.0) / 1024.0)
    occ = room_occupancy(rng_for(seed_block, 3), g, 0.05)
    return _field(
        name="room256" if log2_T == 19 else f"room256_T{log2_T}", n_levels=L, log2_T=log2_T,
        level_res=level_resolutions(L, s, f64), base_res=s, growth=f,
        tables=make_tables(rng_for(seed_block, 1), L, log2_T, "normal", table_dtype),
        mlp=make_mlp(rng_for(seed_block, 2), L, 4, density_bias(1e-4, 2.3, float(dt))), sh_bands=4,
        occ_res=g, occ_bits=pack_bits(occ), aabb_min=[0.0, 0.0, 0.0], extent=1.0,
        dt=dt, max_samples=1024, t_min=1e-4, lod_enable=1)


def field_blobs_3m2(table_dtype=np.float16) -> dict:
    """The blob field with its AABB scaled to a 3.2 m cube, FP16 tables."""
    fld = field_blobs64(extent=3.2, table_dtype=table_dtype)
    fld["name"] = "blobs_3m2"
    return fld


def walkable_occupancy(rng, g: int, extent: float, path_xy: np.ndarray,
                       frac: float = 0.03) -> np.ndarray:
    """16 m cube, z-up: floor, ceiling at 3 m, exterior and interior walls
    (4-6 rooms with doorways) and solid furniture, kept clear of the walk."""
    cell = extent / g
    occ = np.zeros((g, g, g), bool)
    c = lambda m: int(round(m / cell))  # metres -> cells
    zc = c(3.0)
    occ[0:2] = True                       # floor slab (2 cells)
    occ[zc:zc + 2] = True                 # ceiling slab
    occ[:zc, :, 0:2] = occ[:zc, :, g - 2:g] = True
    occ[:zc, 0:2, :] = occ[:zc, g - 2:g, :] = True

    def clear_of_path(axis, pos_m, margin=0.7):
        return np.all(np.abs(path_xy[:, axis] - pos_m) > margin)

    def wall(axis, pos_m, lo_m, hi_m):
        p, lo, hi = c(pos_m), c(lo_m), c(hi_m)
        door = rng.uniform(lo_m + 0.5, hi_m - 1.5)
        d0, d1 = c(door), c(door + 1.0)
        if axis == 0:   # wall at x = pos, spanning y in [lo, hi)
            occ[:zc, lo:hi, p:p + 2] = True
            occ[2:c(2.1), d0:d1, p:p + 2] = False
        else:           # wall at y = pos, spanning x in [lo, hi)
            occ[:zc, p:p + 2, lo:hi] = True
            occ[2:c(2.1), p:p + 2, d0:d1] = False

    # one split along x, then each half split along y once or twice -> 4-6 rooms
    for _ in range(100):
        xs = rng.uniform(5.5, 10.5)
        if clear_of_path(0, xs):
            break
    wall(0, xs, 0.0, extent)
    for (x_lo, x_hi) in ((0.0, xs), (xs, extent)):
        n_split = rng.integers(1, 3)
        cuts = []
        for _ in range(n_split):
            for _ in range(100):
                ys = rng.uniform(3.0, 13.0)
                if clear_of_path(1, ys) and all(abs(ys - q) > 2.5 for q in cuts):
                    cuts.append(ys)
                    break
        for ys in cuts:
            wall(1, ys, x_lo, x_hi)

    # solid furniture boxes on the floor until the target fraction is reached
    target = frac * g ** 3
    total = occ.sum()
    while total < target:
        sx, sy = rng.uniform(0.4, 2.0, size=2)
        sz = rng.uniform(0.4, 1.2)
        x0, y0 = rng.uniform(0.1, extent - 0.1 - sx), rng.uniform(0.1, extent - 0.1 - sy)
        # keep a 0.5 m corridor around the walk
        px, py = path_xy[:, 0], path_xy[:, 1]
        dx = np.maximum(np.maximum(x0 - px, px - (x0 + sx)), 0.0)
        dy = np.maximum(np.maximum(y0 - py, py - (y0 + sy)), 0.0)
        if np.min(np.hypot(dx, dy)) < 0.5:
            continue
        blk = occ[2:2 + c(sz), c(y0):c(y0 + sy), c(x0):c(x0 + sx)]
        total += blk.size - blk.sum()
        blk[...] = True
    return occ


def head_path_house(n_frames: int = 300, extent: float = 16.0):
    """300 frames on a 72 Hz timebase: 0.5 m/s walk along the heading, yaw
    rate jitter of +-30 deg/s (smooth, seeded), eye height 1.6 m."""
    rng = rng_for(4, 4)
    dtf = 1.0 / 72.0
    ts = np.arange(n_frames) * dtf
    # smooth yaw-rate: a few random sinusoids scaled to peak 30 deg/s
    w = np.zeros_like(ts)
    for _ in range(4):
        w += rng.uniform(-1, 1) * np.sin(2 * math.pi * rng.uniform(0.1, 0.6) * ts + rng.uniform(0, 2 * math.pi))
    w = w / max(1e-9, np.abs(w).max()) * math.radians(30.0)
    yaw = rng.uniform(0, 2 * math.pi) + np.cumsum(w) * dtf
    start = rng.uniform(6.0, 10.0, size=2)
    step = 0.5 * dtf * np.stack([np.cos(yaw), np.sin(yaw)], axis=1)
    xy = start + np.cumsum(step, axis=0) - step[0]
    return xy, yaw


def field_house512(table_dtype=np.float16) -> dict:
    """Stereo VR scene: 16 m cube, 16 levels, T=2^22, 512^3 bitfield (~3 %)."""
    L, log2_T, s, f = 16, 22, 128.0, 1.4
    g, extent = 512, 16.0
    dt = np.float32(extent * math.sqrt(3.0) / 2048.0)
    xy, _ = head_path_house(300, extent)
    occ = walkable_occupancy(rng_for(4, 3), g, extent, xy, 0.03)
    return _field(
        name="house512", n_levels=L, log2_T=log2_T, level_res=level_resolutions(L, s, f),
        base_res=s, growth=f, tables=make_tables(rng_for(4, 1), L, log2_T, "normal", table_dtype),
        mlp=make_mlp(rng_for(4, 2), L, 4, density_bias(1e-4, 4.6, float(dt))), sh_bands=4,
        occ_res=g, occ_bits=pack_bits(occ), aabb_min=[0.0, 0.0, 0.0], extent=extent,
        dt=dt, max_samples=2048, t_min=1e-4, lod_enable=1)


def field_unbounded(table_dtype=np.float32) -> dict:
    """Unbounded scene for the L-infinity contraction: a room in the inner
    cube (radius 2 m around the origin, 1-cell walls with window openings and
    furniture boxes) and far-field structure beyond it -- a ground band and a
    distant shell -- laid out directly in the contracted cube [-2, 2]^3
    (256^3 cells).  Exponential step schedule beyond 256 steps."""
    L, log2_T, s, nmax = 16, 19, 16.0, 4096.0
    f64 = (nmax / s) ** (1.0 / (L - 1))
    g = 256
    rng = rng_for(6, 3)
    occ = np.zeros((g, g, g), bool)
    lo, hi = g // 4, 3 * g // 4            # inner cube [-1, 1] in contracted units
    occ[lo, lo:hi, lo:hi] = occ[hi - 1, lo:hi, lo:hi] = True          # floor / ceiling (z)
    occ[lo:hi, lo, lo:hi] = occ[lo:hi, hi - 1, lo:hi] = True          # walls (y)
    occ[lo:hi, lo:hi, lo] = occ[lo:hi, lo:hi, hi - 1] = True          # walls (x)
    for _ in range(6):                      # window openings in the walls
        a, b = rng.integers(lo + 10, hi - 40, size=2)
        w = rng.integers(12, 30)
        side = rng.integers(4)
        if side == 0:
            occ[a:a + w, lo, b:b + w] = False
        elif side == 1:
            occ[a:a + w, hi - 1, b:b + w] = False
        elif side == 2:
            occ[a:a + w, b:b + w, lo] = False
        else:
            occ[a:a + w, b:b + w, hi - 1] = False
    for _ in range(12):                     # furniture boxes on the floor
        sx, sy, sz = rng.integers(6, 24, size=3)
        x0, y0 = rng.integers(lo + 2, hi - 2 - 24, size=2)
        occ[lo + 1:lo + 1 + sz, y0:y0 + sy, x0:x0 + sx] = True
    c = (np.arange(g) + 0.5) / g * 4.0 - 2.0
    z, y, x = np.meshgrid(c, c, c, indexing="ij")
    m = np.maximum(np.maximum(np.abs(x), np.abs(y)), np.abs(z))
    occ |= (m > 1.0) & (z > -1.05) & (z < -1.0)                       # ground band
    occ |= m > 1.9                                                     # distant shell
    dt = np.float32(2.0 * math.sqrt(3.0) / 1024.0)   # world step inside the 4 m room
    f = _field(
        name="unbounded", n_levels=L, log2_T=log2_T, level_res=level_resolutions(L, s, f64),
        base_res=s, growth=float(np.float32(f64)),
        tables=make_tables(rng_for(6, 1), L, log2_T, "normal", table_dtype),
        mlp=make_mlp(rng_for(6, 2), L, 4, density_bias(1e-4, 2.3, float(dt))), sh_bands=4,
        occ_res=g, occ_bits=pack_bits(occ), aabb_min=[-2.0, -2.0, -2.0], extent=4.0,
        dt=dt, max_samples=1024, t_min=1e-4, lod_enable=1)
    f.update(contraction=1, center=np.zeros(3, np.float32), radius=2.0,
             inv_radius=float(np.float32(1.0 / 2.0)), step_growth=float(np.float32(1.0 / 256.0)),
             max_lattice=1600)
    return f


def field_unbounded_sparse_far(table_dtype=np.float32) -> dict:
    """The unbounded scene's field with other occupancy: the inner cube empty
    and isolated occupied cells (0.2 %) beyond it, so that most occupied
    8-cell blocks of the far field consist of empty 4-cell bricks that rays
    cross before their first hit (inputs for march tests)."""
    f = field_unbounded(table_dtype)
    g = int(f["occ_res"])
    occ = rng_for(6, 5).random((g, g, g)) < 0.002
    c = np.arange(g)
    inner = (c >= g // 4) & (c < 3 * g // 4)
    occ[np.ix_(inner, inner, inner)] = False
    f["occ_bits"] = pack_bits(occ)
    return f


def cameras_unbounded(n=2, W=256, H=256):
    rng = rng_for(6, 4)
    out = []
    for _ in range(n):
        xy = rng.uniform(-1.2, 1.2, 2)
        yaw = rng.uniform(0, 2 * math.pi)
        out.append(camera(look_rotation(yaw, math.radians(rng.uniform(-10, 20))),
                          np.array([xy[0], xy[1], -0.4]), W, H, 90.0))
    return out


def field_serving_room() -> dict:
    """Serving scene C: the room field's architecture with T=2^20 and FP16 tables."""
    return field_room256(log2_T=20, table_dtype=np.float16, seed_block=5)


# ----------------------------------------------------------------------------
# cameras
# ----------------------------------------------------------------------------

def focal_for_fov(size: int, fov_deg: float) -> float:
    return (size / 2.0) / math.tan(math.radians(fov_deg) / 2.0)


def camera(R: np.ndarray, pos: np.ndarray, W: int, H: int, fov_deg: float) -> dict:
    fx = focal_for_fov(W, fov_deg)
    c2w = np.concatenate([np.asarray(R, np.float64), np.asarray(pos, np.float64)[:, None]], axis=1)
    return {"c2w": c2w.astype(np.float32), "fx": np.float32(fx), "fy": np.float32(fx),
            "cx": np.float32(W / 2.0), "cy": np.float32(H / 2.0)}


def random_rotation(rng) -> np.ndarray:
    q = rng.standard_normal(4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
        [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
        [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)]])


def look_rotation(yaw: float, pitch: float = 0.0) -> np.ndarray:
    """c2w rotation for a z-up world: columns = (right, down, forward)."""
    fwd = np.array([math.cos(pitch) * math.cos(yaw), math.cos(pitch) * math.sin(yaw), math.sin(pitch)])
    right = np.array([math.sin(yaw), -math.cos(yaw), 0.0])
    down = np.cross(fwd, right)
    return np.stack([right, down, fwd], axis=1)


def cameras_blobs64(n: int = 1, W: int = 64, H: int = 64, seed_part: int = 4):
    rng = rng_for(1, seed_part)
    return [camera(random_rotation(rng), rng.uniform(0.2, 0.8, 3), W, H, 60.0) for _ in range(n)]


def cameras_room256(n: int = 1, W: int = 1024, H: int = 1024, seed_block: int = 2):
    rng = rng_for(seed_block, 4)
    cams = []
    for _ in range(n):
        xy = rng.uniform(0.2, 0.8, 2)
        yaw = rng.uniform(0, 2 * math.pi)
        pitch = math.radians(rng.uniform(-15, 15))
        cams.append(camera(look_rotation(yaw, pitch), np.array([xy[0], xy[1], 0.5]), W, H, 90.0))
    return cams


def cameras_walk_3m2(n: int = 32, W: int = 2048, H: int = 2048):
    """n poses along a seeded walk around the 3.2 m field: 3 cm steps on an
    arc of radius 1.1 m about the cube's vertical centre line, facing the
    centre with a smoothly varying yaw offset (a random walk of +-2 degrees
    per step, kept within +-15), eye height 1.6 m +- 0.05."""
    rng = rng_for(3, 4)
    centre = np.array([1.6, 1.6])
    radius = 1.1
    phi = rng.uniform(0, 2 * math.pi)
    off = 0.0
    cams = []
    for i in range(n):
        phi += 0.03 / radius
        off = float(np.clip(off + math.radians(rng.uniform(-2, 2)), -math.radians(15), math.radians(15)))
        p = centre + radius * np.array([math.cos(phi), math.sin(phi)])
        yaw = phi + math.pi + off                      # towards the centre, plus the offset
        z = 1.6 + rng.uniform(-0.05, 0.05)
        cams.append(camera(look_rotation(yaw, 0.0), np.array([p[0], p[1], z]), W, H, 60.0))
    return cams


def stereo_pair(R: np.ndarray, head: np.ndarray, W: int, H: int, fov_deg: float, ipd: float = 0.064):
    """Two parallel-axis eyes at head +- R (ipd/2, 0, 0), computed in FP64 and
    rounded once to FP32."""
    R = np.asarray(R, np.float64)
    off = R @ np.array([ipd / 2.0, 0.0, 0.0])
    return [camera(R, head - off, W, H, fov_deg), camera(R, head + off, W, H, fov_deg)]


def cameras_house_stereo(frames=None, W: int = 2048, H: int = 2048):
    """Stereo pairs along the 300-frame head path: list of [left, right]."""
    xy, yaw = head_path_house(300, 16.0)
    frames = range(300) if frames is None else frames
    out = []
    for i in frames:
        R = look_rotation(float(yaw[i]), 0.0)
        head = np.array([xy[i, 0], xy[i, 1], 1.6])
        out.append(stereo_pair(R, head, W, H, 100.0))
    return out


def fields_serving():
    a = field_blobs64()
    a["name"] = "serving_blobs64"
    b = field_blobs_3m2()
    b["name"] = "serving_blobs_3m2"
    c = field_serving_room()
    c["name"] = "serving_room256_T20"
    return {"A": a, "B": b, "C": c}


def serving_requests(n: int, rate_hz: float, seed: int = 5004):
    """Poisson arrivals; mix 40 % 256^2, 40 % 1024^2, 20 % 2x2048^2 stereo;
    scene uniform over A, B, C."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate_hz, size=n)
    t = np.cumsum(gaps) - gaps[0]
    reqs = []
    for i in range(n):
        u = rng.uniform()
        kind = "preview" if u < 0.4 else ("tile" if u < 0.8 else "stereo")
        scene = "ABC"[rng.integers(3)]
        reqs.append({"t": float(t[i]), "kind": kind, "scene": scene,
                     "pose_seed": int(rng.integers(1 << 30))})
    return reqs


def request_cameras(scene: str, kind: str, pose_seed: int):
    rng = np.random.default_rng(pose_seed)
    W = {"preview": 256, "tile": 1024, "stereo": 2048}[kind]
    if scene == "C":
        xy = rng.uniform(0.2, 0.8, 2)
        R = look_rotation(rng.uniform(0, 2 * math.pi), math.radians(rng.uniform(-15, 15)))
        pos, fov = np.array([xy[0], xy[1], 0.5]), 90.0
    elif scene == "B":
        R = look_rotation(rng.uniform(0, 2 * math.pi), 0.0)
        pos, fov = np.array([rng.uniform(0.8, 2.4), rng.uniform(0.8, 2.4), 1.6]), 60.0
    else:
        R = random_rotation(rng)
        pos, fov = rng.uniform(0.2, 0.8, 3), 60.0
    if kind == "stereo":
        ipd = 0.064 if scene == "B" else 0.02
        return stereo_pair(R, pos, W, W, fov, ipd), W, W
    return [camera(R, pos, W, W, fov)], W, W


# ----------------------------------------------------------------------------
# field files: <prefix>.npz (arrays) + <prefix>.json (scalars), no pickles
# ----------------------------------------------------------------------------

_SCALARS = ("name", "n_levels", "log2_T", "n_feat", "base_res", "growth", "sh_bands",
            "occ_res", "extent", "dt", "max_samples", "t_min", "lod_enable", "lod_bias",
            "lod_radius_scale", "contraction", "radius", "inv_radius", "step_growth", "max_lattice")


def save_field(prefix: str, field: dict) -> None:
    arrays = {"level_res": field["level_res"], "hash_primes": field["hash_primes"],
              "tables": field["tables"], "occ_bits": field["occ_bits"],
              "aabb_min": field["aabb_min"]}
    for k, v in field["mlp"].items():
        arrays["mlp_" + k] = v
    np.savez(prefix + ".npz", **arrays)
    meta = {k: (field[k].item() if hasattr(field[k], "item") else field[k]) for k in _SCALARS if k in field}
    if "center" in field:
        meta["center"] = [float(v) for v in np.asarray(field["center"], np.float32)]
    meta["format"] = "vrn-field-1"
    meta["table_dtype"] = str(np.dtype(field["tables"].dtype))
    meta["sh_convention"] = "real, no Condon-Shortley phase, bands 0..n-1, order (l, m=-l..l)"
    with open(prefix + ".json", "w") as fh:
        json.dump(meta, fh, indent=1)


def field_bytes(field: dict) -> int:
    return int(field["tables"].nbytes + field["occ_bits"].nbytes
               + sum(v.nbytes for v in field["mlp"].values()))
