"""The whole per-pixel pipeline of the renderer hot path, FP64 -- Sec. 4-5:
rays -> dense-masked occupancy march -> LOD hash encoding -> density MLP ->
SH of the direction -> color MLP (sigmoid, PQ units) -> front-to-back
compositing with early termination.  Optionally decoded to linear HDR
(Sec. 4.1: linear 1 = 100 cd/m^2).

This is the plain definition: every lattice sample of every ray is visited
and tested, every stage is computed in FP64 (discrete cell decisions on the
canonical FP32 geometry), no blocking or reordering beyond vectorising over
rays.
"""
import numpy as np

from . import composite as comp
from .encoding import encode, level_star, lod_weights
from .geometry import contract64, is_contracted, lattice_table, pipeline_field
from .march import dense_masked_march, sample_points, uses_table
from .mlp import color_mlp, density_mlp
from .pq import pq_to_linear
from .rays import canonical_rays, cone_pitch, fp64_directions
from .sh import sh_basis


def all_pixels(n_cams, W, H, rows=None, cols=None):
    """Pixel list (camera, row, col) in framebuffer order; no passage."""
    rows = np.arange(H) if rows is None else np.asarray(rows)
    cols = np.arange(W) if cols is None else np.asarray(cols)
    c, r, x = np.meshgrid(np.arange(n_cams), rows, cols, indexing="ij")
    return np.stack([c.ravel(), r.ravel(), x.ravel()], axis=1)


def contracted_level_star(field, cam, cols, rows, o, t):
    """L* from the footprint between corresponding sample points of adjacent
    rays in contracted space (Sec. 4.2.1), FP64, normalised by the cube edge 4."""
    d0 = fp64_directions(cam, cols, rows)
    d1 = fp64_directions(cam, np.asarray(cols) + 1, rows)
    o64 = np.asarray(o, np.float64)
    t = np.asarray(t, np.float64)[:, None]
    y0 = contract64(o64 + t * d0, field)
    y1 = contract64(o64 + t * d1, field)
    rhat = float(field.get("lod_radius_scale", 1.0)) * np.linalg.norm(y1 - y0, axis=-1) / 4.0
    s = np.float64(np.float32(field["base_res"]))
    f = np.float64(np.float32(field["growth"]))
    ls = -np.log(2.0 * s * rhat) / np.log(f) + np.float64(np.float32(field["lod_bias"]))
    return np.maximum(ls, 0.0)


def _render_batch(field, cam, rows, cols, band, rank_block, keep_k):
    """Sec. 4-5 per-pixel pipeline for one batch of pixels of one camera."""
    o, d = canonical_rays(cam, cols, rows)
    n = o.shape[0]
    lod = bool(field["lod_enable"])
    contracted = is_contracted(field)
    pf = pipeline_field(field)
    deltas = lattice_table(field)[1] if uses_table(field) else None
    r = cone_pitch(cam, cols, rows, float(field["lod_radius_scale"])) if lod and not contracted else None
    ks, counts = dense_masked_march(field, o, d)
    sh = sh_basis(d.astype(np.float64), int(field["sh_bands"]))
    st = comp.new_state(n)
    L = int(field["n_levels"])
    m = int(counts.max(initial=0))
    for r0 in range(0, m, rank_block):
        live = np.nonzero((counts > r0) & ~st["hi_done"])[0]
        if live.size == 0:
            break
        ranks = np.arange(r0, min(r0 + rank_block, m))
        rr, jj = np.meshgrid(live, ranks, indexing="ij")
        ok = jj < counts[rr]
        rr, jj = rr[ok], jj[ok]
        k = ks[rr, jj]
        x, tk = sample_points(field, o[rr], d[rr], k[:, None])
        x, tk = x[:, 0, :], tk[:, 0]
        if lod and contracted:
            w = lod_weights(contracted_level_star(field, cam, cols[rr], rows[rr], o[rr], tk), L)
        elif lod:
            w = lod_weights(level_star(tk.astype(np.float64), r[rr], field), L)
        else:
            w = np.ones((rr.size, L))
        step_len = deltas[k] if deltas is not None else np.full(k.size, np.float32(field["dt"]))
        feats = encode(pf, x, w)
        sigma, geo = density_mlp(feats, field["mlp"])
        rgb = color_mlp(geo, sh[rr], field["mlp"])
        nlev = (w > 0).sum(axis=1)
        for j in ranks:
            sel = jj == j
            rows_j = rr[sel]
            keep = ~st["hi_done"][rows_j]
            if not keep.any():
                continue
            idx = np.nonzero(sel)[0][keep]
            comp.step(st, rr[idx], sigma[idx], rgb[idx], step_len[idx], float(field["t_min"]),
                      band, nlev[idx])
    comp.finish(st)
    out = {
        "rgba": np.concatenate([st["star_C"], 1.0 - st["star_T"][:, None]], axis=1),
        "n": st["star_n"],
        "rgba_lo": np.concatenate([st["lo_C"], 1.0 - st["lo_T"][:, None]], axis=1),
        "n_lo": st["lo_n"],
        "rgba_hi": np.concatenate([st["hi_C"], 1.0 - st["hi_T"][:, None]], axis=1),
        "n_hi": st["hi_n"],
        "levels": st["levels"],
    }
    if keep_k:
        out["ks"] = [ks[i, :counts[i]].copy() for i in range(n)]
    return out


def render_fp64(field, cams, W, H, pixels=None, band=1e-4, batch=4096, rank_block=8,
                keep_k=False, linear_hdr=False):
    """Render pixels [m, 3] of (camera, row, col) (default: every pixel).

    Returns a dict of arrays over the m pixels: rgba (PQ RGB + alpha) at the
    FP64 termination rule, n (composited samples), the tie-range ends
    rgba_lo/n_lo and rgba_hi/n_hi, tie (bool), levels (hash levels read
    summed over the composited samples) and, with keep_k, the evaluated
    lattice indices per pixel (uncapped by termination).
    Sec. 4-5: march (4.3), LOD hash encoding (4.2.1), MLPs (6), compositing (4.1)."""
    if pixels is None:
        pixels = all_pixels(len(cams), W, H)
    pixels = np.asarray(pixels, np.int64)
    m = pixels.shape[0]
    res = {"rgba": np.zeros((m, 4)), "n": np.zeros(m, np.int64),
           "rgba_lo": np.zeros((m, 4)), "n_lo": np.zeros(m, np.int64),
           "rgba_hi": np.zeros((m, 4)), "n_hi": np.zeros(m, np.int64),
           "levels": np.zeros(m, np.int64)}
    ks_all = [None] * m if keep_k else None
    for ci, cam in enumerate(cams):
        sel_c = np.nonzero(pixels[:, 0] == ci)[0]
        for b0 in range(0, sel_c.size, batch):
            sel = sel_c[b0:b0 + batch]
            out = _render_batch(field, cam, pixels[sel, 1], pixels[sel, 2], band, rank_block, keep_k)
            for key in res:
                res[key][sel] = out[key]
            if keep_k:
                for a, i in enumerate(sel):
                    ks_all[i] = out["ks"][a]
    res["tie"] = res["n_lo"] != res["n_hi"]
    if linear_hdr:
        for key in ("rgba", "rgba_lo", "rgba_hi"):
            res[key][:, :3] = pq_to_linear(res[key][:, :3])
    if keep_k:
        res["ks"] = ks_all
    return res
