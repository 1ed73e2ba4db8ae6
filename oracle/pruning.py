"""Grid-based occupancy pruning, FP64 -- Sec. 4.3 (the grid half of the
joint history and grid pruning) and App. C (the pruning ablation).

Grid pruning estimates the maximum density inside each occupancy voxel by
evaluating the density MLP on points placed evenly inside it (the paper uses
4 points per voxel), converts it to an opacity with the worst-case (minimum)
step, and prunes the voxel when that opacity falls below the threshold
alpha (annealed to 0.2 in the paper).  History pruning needs training and is
out of scope; the grid estimate alone decides here.

Readings:
* "4 points ... evenly placed": the four alternating corners of a 2x2x2
  sub-lattice of the voxel, at offsets {1/4, 3/4} with an even number of
  3/4's (a regular tetrahedron); a p^3 pattern at offsets (i + 1/2)/p is the
  general "dense cubic grid".
* the renderer's lattice is uniform, so the worst-case step is dt and the
  opacity is 1 - exp(-sigma_max dt);
* densities are evaluated with every hash level (no ray, hence no LOD);
* pruning only clears bits: out = in AND (opacity_max >= alpha).
* sample points are canonical FP32 positions
  x = aabb_min + ((float)c + offset) * cell, cell = fp32(extent / G), each op
  rounded; the encoding then proceeds in FP64 as in the renderer.
"""
import numpy as np

from .encoding import encode
from .mlp import density_mlp

F32 = np.float32


def voxel_offsets(points_per_voxel):
    """App. C, four evenly placed points per voxel (reading R29)."""
    if points_per_voxel == 4:
        q, t = 0.25, 0.75
        return np.array([[q, q, q], [t, t, q], [t, q, t], [q, t, t]], F32)
    p = int(round(points_per_voxel ** (1.0 / 3.0)))
    if p ** 3 != points_per_voxel:
        raise ValueError("points_per_voxel must be 4 or a cube")
    g = (np.arange(p) + 0.5) / p
    z, y, x = np.meshgrid(g, g, g, indexing="ij")
    return np.stack([x.ravel(), y.ravel(), z.ravel()], -1).astype(F32)


def voxel_points(field, cells, offsets):
    """Canonical FP32 points [n_vox, n_pts, 3] for integer cells [n_vox, 3].
    Sec. 4.3 and App. C; reading R29."""
    G = int(field["occ_res"])
    cell = F32(np.float64(F32(field["extent"])) / np.float64(G))
    amin = np.asarray(field["aabb_min"], F32)
    c = cells.astype(F32)[:, None, :]
    return (amin[None, None, :] + (c + offsets[None, :, :]) * cell).astype(F32)


def grid_prune_fp64(field, alpha, points_per_voxel=4, band=1e-5, batch=65536, voxels=None):
    """Returns (bits_out uint32 words, max_opacity [G^3] float64 (NaN where the
    voxel was not occupied or not evaluated), tie [G^3] bool: |opacity - alpha|
    <= band*alpha).  ``voxels`` restricts the evaluation to a subset of linear
    voxel indices (bits outside it are then meaningless).
    Sec. 4.3 grid pruning with App. C's points; reading R29."""
    G = int(field["occ_res"])
    bits = np.asarray(field["occ_bits"], np.uint32)
    n = G ** 3
    idx = np.arange(n, dtype=np.int64)
    occ = ((bits[idx >> 5] >> (idx & 31).astype(np.uint32)) & 1).astype(bool)
    vox = np.nonzero(occ)[0]
    if voxels is not None:
        vox = np.intersect1d(vox, np.asarray(voxels, np.int64))
    offsets = voxel_offsets(points_per_voxel)
    dt = np.float64(F32(field["dt"]))
    max_op = np.full(n, np.nan)
    for b0 in range(0, vox.size, batch):
        v = vox[b0:b0 + batch]
        cells = np.stack([v % G, (v // G) % G, v // (G * G)], -1)
        pts = voxel_points(field, cells, offsets).reshape(-1, 3)
        sigma, _ = density_mlp(encode(field, pts), field["mlp"])
        op = 1.0 - np.exp(-sigma * dt)
        max_op[v] = op.reshape(v.size, -1).max(axis=1)
    keep = occ & (np.nan_to_num(max_op, nan=-1.0) >= alpha)
    pad = (-n) % 32
    out = np.packbits(np.concatenate([keep, np.zeros(pad, bool)]).astype(np.uint8), bitorder="little")
    words = out.view("<u4").astype(np.uint32)
    tie = occ & (np.abs(np.nan_to_num(max_op, nan=-1.0) - alpha) <= band * alpha)
    return words, max_op, tie
