"""Per-pixel rays -- Sec. 4.2.1 (cone base radius) and the pinhole model.

Discrete decisions (which lattice samples fall in which occupancy cell) are
taken on a canonical FP32 ray so that "bit-exact cell indices" is well
defined; every continuous quantity is FP64.

Canonical FP32 ray for pixel (i = column, j = row), every operation rounded
to FP32 and no fused multiply-add:
    a = ((i + 0.5) - cx) / fx,  b = ((j + 0.5) - cy) / fy
    w_r = (R[r,0]*a + R[r,1]*b) + R[r,2]            (r = x, y, z)
    n = sqrt((w_x*w_x + w_y*w_y) + w_z*w_z),  d = w / n
    o = translation column of the camera-to-world matrix.
Axes follow OpenCV (+x right, +y down, +z forward), pixel centres at +0.5.

Cone pitch (Sec. 4.2.1): the base radius r at unit distance is read as the
spacing of corresponding unit-distance points on adjacent rays,
r = scale * || dir(i+1, j) - dir(i, j) ||, with dir the FP64 unit direction.
"""
import numpy as np

F32 = np.float32


def canonical_rays(cam, i, j):
    """FP32 origins and unit directions for integer pixel arrays i (col), j (row).
    Reading R20 (camera model) and R13 (canonical FP32 order)."""
    c2w = np.asarray(cam["c2w"], F32)
    fx, fy, cx, cy = (F32(cam[k]) for k in ("fx", "fy", "cx", "cy"))
    fi = np.asarray(i).astype(F32) + F32(0.5)
    fj = np.asarray(j).astype(F32) + F32(0.5)
    a = (fi - cx) / fx
    b = (fj - cy) / fy
    w = [(c2w[r, 0] * a + c2w[r, 1] * b) + c2w[r, 2] for r in range(3)]
    n = np.sqrt((w[0] * w[0] + w[1] * w[1]) + w[2] * w[2])
    d = np.stack([w[0] / n, w[1] / n, w[2] / n], axis=-1).astype(F32)
    o = np.broadcast_to(c2w[:, 3], d.shape).astype(F32)
    return o, d


def fp64_directions(cam, i, j):
    """Exact-arithmetic (FP64) unit ray directions.  Reading R20 (camera model), in FP64."""
    c2w = np.asarray(cam["c2w"], F32).astype(np.float64)
    fx, fy, cx, cy = (np.float64(F32(cam[k])) for k in ("fx", "fy", "cx", "cy"))
    a = (np.asarray(i, np.float64) + 0.5 - cx) / fx
    b = (np.asarray(j, np.float64) + 0.5 - cy) / fy
    w = np.stack([a, b, np.ones_like(a)], axis=-1) @ c2w[:, :3].T
    return w / np.linalg.norm(w, axis=-1, keepdims=True)


def cone_pitch(cam, i, j, scale=1.0):
    """Base radius at unit distance: distance between the unit directions of
    pixel (i, j) and its right neighbour (i + 1, j), FP64.
    Sec. 4.2.1 base radius; reading R5."""
    d0 = fp64_directions(cam, i, j)
    d1 = fp64_directions(cam, np.asarray(i) + 1, j)
    return scale * np.linalg.norm(d1 - d0, axis=-1)
