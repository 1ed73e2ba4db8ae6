"""Shared helpers of the GPU parity tests (not collected by pytest)."""
import math

import numpy as np
import pytest

from paper_2311_02542_amd import synth

F32 = np.float32


def need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    return torch


def tiny_field(g, occ, amin=(0.0, 0.0, 0.0), extent=1.0, dt=None, cap=64, seed=0, L=2,
               log2_T=10, lod=False, bands=2, table_dtype=np.float32, b_sigma=4.0):
    """Small but complete field (random tables / MLP) on a G^3 bitfield."""
    rng = np.random.default_rng(seed)
    res = np.array([max(1, int(4 * 2.1 ** l)) for l in range(L)], np.uint32)
    f = {"name": "tiny", "n_levels": L, "log2_T": log2_T, "n_feat": 2, "level_res": res,
         "hash_primes": np.array(synth.HASH_PRIMES, np.uint32), "base_res": 4.0, "growth": 2.1,
         "tables": rng.uniform(-0.5, 0.5, (L, 1 << log2_T, 2)).astype(table_dtype),
         "mlp": synth.make_mlp(rng, L, bands, b_sigma), "sh_bands": bands, "occ_res": g,
         "occ_bits": synth.pack_bits(np.asarray(occ, bool)),
         "aabb_min": np.array(amin, F32), "extent": float(F32(extent)),
         "dt": float(F32(dt if dt else extent * math.sqrt(3) / (5 * g))), "max_samples": cap,
         "t_min": float(F32(1e-4)), "lod_enable": int(lod), "lod_bias": 0.0, "lod_radius_scale": 1.0}
    return f


def axis_camera(R, pos, W=8, H=8, fx=7.0, cx=0.5, cy=0.5):
    c2w = np.concatenate([np.asarray(R, float), np.asarray(pos, float)[:, None]], 1).astype(F32)
    return {"c2w": c2w, "fx": F32(fx), "fy": F32(fx), "cx": F32(cx), "cy": F32(cy)}


def compare_render(gpu_rgba, gpu_n, ref, tol, mask=None):
    """Check a GPU render against oracle output dict ``ref`` (pixels flattened
    in the same order).  Sample counts must be bit-exact, except on tie pixels
    where any count in [n_lo, n_hi] is accepted; colors must be within ``tol``
    of the oracle result at the matching termination point."""
    g_rgba = np.asarray(gpu_rgba, np.float64).reshape(-1, 4)
    g_n = np.asarray(gpu_n).reshape(-1).astype(np.int64)
    if mask is not None:
        g_rgba, g_n = g_rgba[mask], g_n[mask]
    tie = ref["tie"]
    ok_n = np.where(tie, (g_n >= ref["n_lo"]) & (g_n <= ref["n_hi"]), g_n == ref["n"])
    bad = np.nonzero(~ok_n)[0]
    assert bad.size == 0, f"{bad.size} sample-count mismatches, e.g. px {bad[:5]}: gpu {g_n[bad[:5]]} oracle {ref['n'][bad[:5]]}"
    want = np.where((tie & (g_n == ref["n_lo"]))[:, None], ref["rgba_lo"],
                    np.where((tie & (g_n == ref["n_hi"]))[:, None], ref["rgba_hi"], ref["rgba"]))
    err = np.abs(g_rgba - want)
    # a tie pixel stopped strictly between the two ends: compositing only
    # adds non-negative terms, so every channel lies between its values at
    # n_lo and n_hi; the error is the distance outside that interval
    mid = tie & (g_n != ref["n_lo"]) & (g_n != ref["n_hi"])
    lo = np.minimum(ref["rgba_lo"][mid], ref["rgba_hi"][mid])
    hi = np.maximum(ref["rgba_lo"][mid], ref["rgba_hi"][mid])
    err[mid] = np.maximum(np.maximum(lo - g_rgba[mid], g_rgba[mid] - hi), 0.0)
    return float(err.max(initial=0.0)), float(err.mean() if err.size else 0.0), int(tie.sum())
