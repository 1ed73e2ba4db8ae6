"""Sample geometry of a field: where lattice sample k of a ray lies, its step
length, and the coordinates the occupancy grid and the hash grid see.

Two kinds of fields:

* bounded (the default): the cube [aabb_min, aabb_min + extent]; uniform
  lattice t_k = (k + 1/2) dt (reading R11); delta_k = dt.

* unbounded, with the L-infinity cubic contraction of Sec. 4 (after the
  paper's contraction reference; used for its far-field scenes): with
  u = (x - center) * inv_radius and m = max_i |u_i|,
      C(u) = u                        if m <= 1
      C(u) = (2 - 1/m) (u / m)        otherwise,
  so all of space maps into the cube [-2, 2]^3, which plays the role of the
  field's AABB (aabb_min = -2, extent = 4) for occupancy and hashing.
  Samples follow an exponential-distance schedule (Sec. 6: exponential
  distances; reading R30): a canonical FP32 table
      t_0 = dt / 2,  t_{k+1} = t_k + max(dt, growth * t_k)
  with every operation rounded to FP32, and delta_k = t_{k+1} - t_k.
  The canonical contracted position of a sample, each op rounded to FP32:
      x = o + t_k d;  u = (x - center) * inv_radius;  m = max |u|;
      y = u if m <= 1 else u * ((2 - 1/m) * (1/m)).
  The LOD footprint is measured directly between corresponding sample
  points of adjacent rays in contracted space (Sec. 4.2.1): r_hat_n =
  |C(u(i+1, j)) - C(u(i, j))| / 4 in normalised units, FP64.
"""
import numpy as np

F32 = np.float32


def is_contracted(field):
    """Whether the field uses the L-infinity contraction (Sec. 4; reading R31)."""
    return bool(field.get("contraction", 0))


def lattice_table(field):
    """Canonical FP32 sample distances t_k (k < max_lattice) and steps.
    Sec. 6 exponential sample distances; reading R30."""
    dt = F32(field["dt"])
    growth = F32(field.get("step_growth", 0.0))
    K = int(field["max_lattice"])
    t = np.empty(K + 1, F32)
    t[0] = F32(0.5) * dt
    for k in range(K):
        t[k + 1] = F32(t[k] + max(dt, F32(growth * t[k])))
    return t[:K], (t[1:] - t[:K]).astype(F32)


def pipeline_field(field):
    """The field as the occupancy / hash stages see it: contracted fields use
    the cube [-2, 2]^3 as their AABB.
    Sec. 4 contraction (reading R31): the grids cover the contracted cube."""
    if not is_contracted(field):
        return field
    f = dict(field)
    f["aabb_min"] = np.array([-2.0, -2.0, -2.0], F32)
    f["extent"] = 4.0
    return f


def contract32(x, field):
    """Canonical FP32 contraction of world points x [..., 3].
    Sec. 4 L-infinity contraction in the canonical FP32 order (reading R31)."""
    c = np.asarray(field["center"], F32)
    ir = F32(field["inv_radius"])
    u = np.stack([(x[..., a] - c[a]) * ir for a in range(3)], axis=-1).astype(F32)
    m = np.max(np.abs(u), axis=-1)
    with np.errstate(divide="ignore"):
        im = (F32(1.0) / m).astype(F32)
    s = ((F32(2.0) - im) * im).astype(F32)
    y = np.where((m <= F32(1.0))[..., None], u, (u * s[..., None]).astype(F32))
    return y.astype(F32)


def contract64(x, field):
    """Sec. 4 L-infinity contraction in FP64 (reading R31)."""
    c = np.asarray(field["center"], F32).astype(np.float64)
    u = (np.asarray(x, np.float64) - c) * np.float64(F32(field["inv_radius"]))
    m = np.max(np.abs(u), axis=-1, keepdims=True)
    return np.where(m <= 1.0, u, (2.0 - 1.0 / m) * u / np.maximum(m, 1e-300))
