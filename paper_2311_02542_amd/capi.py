"""Thin ctypes binding of libvrn.so (include/vrn.h).

Argument marshalling only: every step of the render runs in the library's
HIP kernels.  Device buffers are torch tensors (PyTorch is used for device
memory and streams only); host inputs are the plain field / camera dicts of
``synth``.  If the library is missing this module raises -- there is no CPU
fallback.
"""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libvrn.so")
HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "vrn.h")

VRN_OK, VRN_ERR_INVALID_ARG, VRN_ERR_UNSUPPORTED, VRN_ERR_OUT_OF_MEMORY = 0, -1, -2, -3
VRN_ERR_BUDGET, VRN_ERR_DEVICE, VRN_ERR_NOT_FOUND, VRN_ERR_BUSY = -4, -5, -6, -7
VRN_ERR_TIMEOUT, VRN_ERR_CANCELLED = -8, -9
VRN_F32, VRN_F16, VRN_BF16, VRN_F32X = 0, 1, 2, 3
DTYPES = {"f32": VRN_F32, "f16": VRN_F16, "bf16": VRN_BF16, "f32x": VRN_F32X}
STATUS_NAMES = {0: "VRN_OK", -1: "VRN_ERR_INVALID_ARG", -2: "VRN_ERR_UNSUPPORTED",
                -3: "VRN_ERR_OUT_OF_MEMORY", -4: "VRN_ERR_BUDGET", -5: "VRN_ERR_DEVICE",
                -6: "VRN_ERR_NOT_FOUND", -7: "VRN_ERR_BUSY", -8: "VRN_ERR_TIMEOUT", -9: "VRN_ERR_CANCELLED"}
MAX_CAMS = 16

c_f = ctypes.c_float
c_u32 = ctypes.c_uint32
c_i32 = ctypes.c_int32
c_u64 = ctypes.c_uint64
c_vp = ctypes.c_void_p


class VrnFieldDesc(ctypes.Structure):
    _fields_ = [("n_levels", c_u32), ("log2_T", c_u32), ("n_feat", c_u32),
                ("level_res", ctypes.POINTER(c_u32)), ("hash_primes", c_u32 * 3),
                ("base_res", c_f), ("growth", c_f), ("table_dtype", c_i32), ("tables", c_vp),
                ("mlp_in", c_u32), ("mlp_hidden", c_u32), ("geo_out", c_u32), ("sh_bands", c_u32),
                ("weights", ctypes.POINTER(c_f)), ("occ_res", c_u32),
                ("occ_bits", ctypes.POINTER(c_u32)), ("aabb_min", c_f * 3), ("extent", c_f),
                ("dt", c_f), ("max_samples", c_u32), ("t_min", c_f), ("lod_enable", c_i32),
                ("lod_bias", c_f), ("lod_radius_scale", c_f), ("contraction", c_i32),
                ("center", c_f * 3), ("radius", c_f), ("step_growth", c_f), ("max_lattice", c_u32)]


class VrnCamera(ctypes.Structure):
    _fields_ = [("c2w", c_f * 12), ("fx", c_f), ("fy", c_f), ("cx", c_f), ("cy", c_f),
                ("row_begin", c_u32), ("row_end", c_u32)]


class VrnRenderOpts(ctypes.Structure):
    _fields_ = [("compute", c_i32), ("output", c_i32), ("march_budget", c_u32), ("exposure_ev", c_f)]


VRN_OUT_PQ, VRN_OUT_LINEAR, VRN_OUT_SRGB = 0, 1, 2
OUTPUTS = {"pq": VRN_OUT_PQ, "linear": VRN_OUT_LINEAR, "srgb": VRN_OUT_SRGB}


class VrnStats(ctypes.Structure):
    _fields_ = [("rays", c_u64), ("samples", c_u64), ("level_fetches", c_u64),
                ("march_steps", c_u64), ("rounds", c_u64), ("tiles", c_u64)]


class VrnServerOpts(ctypes.Structure):
    _fields_ = [("n_slots", c_u32), ("max_batch", c_u32), ("use_graphs", c_i32), ("render", VrnRenderOpts),
                ("d_arena", c_vp), ("arena_bytes", c_u64)]


VRN_SERVE_RELEASE_ON_DONE = 1


class VrnRequestOpts(ctypes.Structure):
    _fields_ = [("t_arrival", ctypes.c_double), ("timeout_s", ctypes.c_double), ("flags", c_u32)]


class VrnServed(ctypes.Structure):
    _fields_ = [("status", c_i32), ("field", c_u32), ("n_cams", c_u32), ("W", c_u32), ("H", c_u32),
                ("d_rgba", c_vp), ("d_nsamples", c_vp), ("t_arrival", ctypes.c_double),
                ("t_launch", ctypes.c_double), ("t_done", ctypes.c_double)]


class VrnServeStats(ctypes.Structure):
    _fields_ = [(name, c_u64) for name in (
        "arena_bytes", "used_bytes", "held_bytes", "largest_free_bytes", "pending", "running", "requests",
        "buffers", "buckets", "launches", "graph_launches", "merged_requests", "captures", "evictions",
        "completed", "failed")]


class VrnError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


_lib = None


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libvrn.so once; raise if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} not found: build it with paper_2311_02542_amd/build.py "
                           "(there is no CPU fallback)")
    lib = ctypes.CDLL(path)
    P = ctypes.POINTER
    sig = {
        "vrn_create": (c_i32, [ctypes.c_int, c_u64, P(c_vp)]),
        "vrn_destroy": (None, [c_vp]),
        "vrn_last_error": (ctypes.c_char_p, []),
        "vrn_load_field": (c_i32, [c_vp, P(VrnFieldDesc), P(c_u32)]),
        "vrn_unload_field": (c_i32, [c_vp, c_u32]),
        "vrn_field_bytes": (c_i32, [c_vp, c_u32, P(c_u64)]),
        "vrn_workspace_bytes": (c_i32, [c_vp, P(c_u64)]),
        "vrn_workspace_init": (c_i32, [c_vp, c_vp, c_u64, c_vp]),
        "vrn_render_bytes": (c_i32, [c_vp, c_u32, c_u32, c_u32, c_u32, P(VrnRenderOpts), P(c_u64)]),
        "vrn_render": (c_i32, [c_vp, c_u32, P(VrnCamera), c_u32, c_u32, c_u32, P(VrnRenderOpts),
                               c_vp, c_vp, c_vp, c_u64, c_vp]),
        "vrn_render_device_cams": (c_i32, [c_vp, c_u32, c_vp, c_u32, c_u32, c_u32,
                                           P(VrnRenderOpts), c_vp, c_vp, c_vp, c_u64, c_vp]),
        "vrn_render_noalloc": (c_i32, [c_vp, c_u32, c_vp, c_u32, c_u32, c_u32, P(VrnRenderOpts), c_vp,
                                       c_vp, c_vp]),
        "vrn_check_cameras": (c_i32, [P(VrnCamera), c_u32, c_u32, c_u32]),
        "vrn_read_stats": (c_i32, [c_vp, c_vp, P(VrnStats), c_vp]),
        "vrn_rays": (c_i32, [c_vp, P(VrnCamera), c_u32, c_u32, c_u32, c_f, c_vp, c_vp, c_vp, c_vp]),
        "vrn_march": (c_i32, [c_vp, c_u32, P(VrnCamera), c_u32, c_u32, c_u32, c_vp, c_u32, c_vp,
                              c_vp]),
        "vrn_encode": (c_i32, [c_vp, c_u32, c_vp, c_vp, c_vp, c_u32, c_vp, c_vp]),
        "vrn_mlp": (c_i32, [c_vp, c_u32, c_vp, c_vp, c_u32, c_i32, c_vp, c_vp, c_vp]),
        "vrn_prune_grid": (c_i32, [c_vp, c_u32, c_f, c_u32, c_i32, c_vp, c_vp, c_vp]),
        "vrn_set_occupancy": (c_i32, [c_vp, c_u32, c_vp, c_vp]),
        "vrn_debug_counters": (c_i32, [c_vp, P(c_u64), ctypes.c_int]),
        "vrn_phase_cycles": (c_i32, [c_vp, P(c_u64), ctypes.c_int]),
        "vrn_server_create": (c_i32, [c_vp, P(VrnServerOpts), P(c_vp)]),
        "vrn_server_destroy": (None, [c_vp]),
        "vrn_server_hold": (c_i32, [c_vp, ctypes.c_int]),
        "vrn_server_prepare": (c_i32, [c_vp, c_u32, c_u32, c_u32, c_u32]),
        "vrn_server_submit": (c_i32, [c_vp, c_u32, P(VrnCamera), c_u32, c_u32, c_u32, P(VrnRequestOpts),
                                      P(c_u64)]),
        "vrn_server_wait": (c_i32, [c_vp, c_u64, ctypes.c_double, P(VrnServed)]),
        "vrn_server_release": (c_i32, [c_vp, c_u64]),
        "vrn_server_cancel": (c_i32, [c_vp, c_u64]),
        "vrn_server_drain": (c_i32, [c_vp, ctypes.c_double]),
        "vrn_server_evict": (c_i32, [c_vp, c_u32]),
        "vrn_server_stats": (c_i32, [c_vp, P(VrnServeStats)]),
        "vrn_server_clock": (ctypes.c_double, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def header_symbols(path: str = HEADER):
    """Function names the public header declares."""
    txt = open(path).read()
    return sorted(set(re.findall(r"^\s*(?:[\w\s\*]+?)\b(vrn_\w+)\s*\(", txt, re.M)))


def _check(status, lib=None):
    if status != VRN_OK:
        lib = lib or load_library()
        raise VrnError(status, lib.vrn_last_error().decode())


# ---------------------------------------------------------------------------
# marshalling helpers
# ---------------------------------------------------------------------------

def field_weights(field) -> np.ndarray:
    m = field["mlp"]
    parts = [m[k] for k in ("W1", "b1", "W2", "b2", "W3", "b3", "W4", "b4", "W5", "b5")]
    return np.ascontiguousarray(np.concatenate([np.asarray(p, np.float32).ravel() for p in parts]))


def make_field_desc(field):
    """(desc, keepalive) for a field dict."""
    L = int(field["n_levels"])
    level_res = np.ascontiguousarray(field["level_res"], np.uint32)
    tables = np.ascontiguousarray(field["tables"])
    if tables.dtype == np.float32:
        tdt = VRN_F32
    elif tables.dtype == np.float16:
        tdt = VRN_F16
    else:
        raise TypeError("tables must be float32 or float16")
    weights = field_weights(field)
    occ = np.ascontiguousarray(field["occ_bits"], np.uint32)
    d = VrnFieldDesc()
    d.n_levels = L
    d.log2_T = int(field["log2_T"])
    d.n_feat = int(field.get("n_feat", 2))
    d.level_res = level_res.ctypes.data_as(ctypes.POINTER(c_u32))
    d.hash_primes[:] = [int(v) for v in field["hash_primes"]]
    d.base_res = float(field.get("base_res", 1.0))
    d.growth = float(field.get("growth", 2.0))
    d.table_dtype = tdt
    d.tables = tables.ctypes.data
    d.mlp_in = 2 * L
    d.mlp_hidden = 64
    d.geo_out = 16
    d.sh_bands = int(field["sh_bands"])
    d.weights = weights.ctypes.data_as(ctypes.POINTER(c_f))
    d.occ_res = int(field["occ_res"])
    d.occ_bits = occ.ctypes.data_as(ctypes.POINTER(c_u32))
    d.aabb_min[:] = [float(v) for v in np.asarray(field["aabb_min"], np.float32)]
    d.extent = float(field["extent"])
    d.dt = float(field["dt"])
    d.max_samples = int(field["max_samples"])
    d.t_min = float(field["t_min"])
    d.lod_enable = int(bool(field.get("lod_enable", 0)))
    d.lod_bias = float(field.get("lod_bias", 0.0))
    d.lod_radius_scale = float(field.get("lod_radius_scale", 1.0))
    d.contraction = int(field.get("contraction", 0))
    d.center[:] = [float(v) for v in np.asarray(field.get("center", np.zeros(3)), np.float32)]
    d.radius = float(field.get("radius", 1.0))
    d.step_growth = float(field.get("step_growth", 0.0))
    d.max_lattice = int(field.get("max_lattice", 0))
    return d, (level_res, tables, weights, occ)


def make_cameras(cams, H):
    arr = (VrnCamera * len(cams))()
    for i, c in enumerate(cams):
        arr[i].c2w[:] = [float(v) for v in np.asarray(c["c2w"], np.float32).reshape(-1)]
        arr[i].fx, arr[i].fy = float(c["fx"]), float(c["fy"])
        arr[i].cx, arr[i].cy = float(c["cx"]), float(c["cy"])
        arr[i].row_begin = int(c.get("row_begin", 0))
        arr[i].row_end = int(c.get("row_end", H))
    return arr


def _ptr(t):
    """Device pointer of a tensor (or a raw integer address)."""
    if t is None:
        return None
    return ctypes.c_void_p(int(t) if isinstance(t, int) else t.data_ptr())


def _stream(stream):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


# ---------------------------------------------------------------------------
# the C entry points, same names
# ---------------------------------------------------------------------------

def vrn_create(device: int = 0, hbm_budget_bytes: int = 0):
    lib = load_library()
    ctx = c_vp()
    _check(lib.vrn_create(device, hbm_budget_bytes, ctypes.byref(ctx)), lib)
    return ctx


def vrn_destroy(ctx):
    load_library().vrn_destroy(ctx)


def vrn_load_field(ctx, field) -> int:
    lib = load_library()
    d, keep = make_field_desc(field)
    fid = c_u32()
    _check(lib.vrn_load_field(ctx, ctypes.byref(d), ctypes.byref(fid)), lib)
    del keep
    return int(fid.value)


def vrn_unload_field(ctx, fid: int):
    lib = load_library()
    _check(lib.vrn_unload_field(ctx, fid), lib)


def vrn_field_bytes(ctx, fid: int) -> int:
    lib = load_library()
    out = c_u64()
    _check(lib.vrn_field_bytes(ctx, fid, ctypes.byref(out)), lib)
    return int(out.value)


def vrn_workspace_bytes(ctx) -> int:
    lib = load_library()
    out = c_u64()
    _check(lib.vrn_workspace_bytes(ctx, ctypes.byref(out)), lib)
    return int(out.value)


def vrn_render_bytes(ctx, fid, n_cams, W, H, compute="f32") -> int:
    """Device bytes a render of this shape needs beyond the resident field
    (workspace, RGBA framebuffer and sample counts): the admission size."""
    lib = load_library()
    out = c_u64()
    opts = render_opts(compute)
    _check(lib.vrn_render_bytes(ctx, fid, n_cams, W, H, ctypes.byref(opts), ctypes.byref(out)), lib)
    return int(out.value)


def vrn_workspace_init(ctx, workspace, stream=None):
    lib = load_library()
    _check(lib.vrn_workspace_init(ctx, _ptr(workspace), workspace.numel() * workspace.element_size(),
                                  _stream(stream)), lib)


def render_opts(compute="f32", linear_hdr=False, march_budget=0, output=None, exposure_ev=0.0):
    """output: "pq" (default), "linear" or "srgb"; linear_hdr=True is "linear"."""
    o = VrnRenderOpts()
    o.compute = DTYPES[compute] if isinstance(compute, str) else int(compute)
    if output is None:
        output = "linear" if linear_hdr else "pq"
    o.output = OUTPUTS[output] if isinstance(output, str) else int(output)
    o.march_budget = int(march_budget)
    o.exposure_ev = float(exposure_ev)
    return o


def vrn_render(ctx, fid, cams, W, H, rgba, nsamples=None, compute="f32", linear_hdr=False,
               workspace=None, stream=None, march_budget=0, output=None, exposure_ev=0.0):
    """Enqueue a render of host cameras into the device tensors rgba
    [n_cams, H, W, 4] float32 and nsamples [n_cams, H, W] int32 (optional)."""
    lib = load_library()
    arr = make_cameras(cams, H)
    opts = render_opts(compute, linear_hdr, march_budget, output, exposure_ev)
    ws_bytes = 0 if workspace is None else workspace.numel() * workspace.element_size()
    _check(lib.vrn_render(ctx, fid, arr, len(cams), W, H, ctypes.byref(opts), _ptr(rgba),
                          _ptr(nsamples), _ptr(workspace), ws_bytes, _stream(stream)), lib)


def vrn_render_device_cams(ctx, fid, d_cams, n_cams, W, H, rgba, nsamples=None, compute="f32",
                           linear_hdr=False, workspace=None, stream=None, march_budget=0):
    """As vrn_render with cameras already on the device (a uint8 tensor of
    n_cams * sizeof(vrn_camera) bytes); kernels only, graph-capturable."""
    lib = load_library()
    opts = render_opts(compute, linear_hdr, march_budget)
    ws_bytes = 0 if workspace is None else workspace.numel() * workspace.element_size()
    _check(lib.vrn_render_device_cams(ctx, fid, _ptr(d_cams), n_cams, W, H, ctypes.byref(opts),
                                      _ptr(rgba), _ptr(nsamples), _ptr(workspace), ws_bytes,
                                      _stream(stream)), lib)


def vrn_render_noalloc(ctx, fid, d_cams, n_cams, W, H, rgba, nsamples=None, compute="f32",
                       linear_hdr=False, stream=None, march_budget=0):
    """As vrn_render_device_cams, with the render's counters in the library's
    static per-device scratch: the library allocates nothing.  Calls on one
    GPU must not overlap on the device."""
    lib = load_library()
    opts = render_opts(compute, linear_hdr, march_budget)
    _check(lib.vrn_render_noalloc(ctx, fid, _ptr(d_cams), n_cams, W, H, ctypes.byref(opts), _ptr(rgba),
                                  _ptr(nsamples), _stream(stream)), lib)


def vrn_check_cameras(cams, W, H) -> int:
    lib = load_library()
    arr = make_cameras(cams, H)
    return int(lib.vrn_check_cameras(arr, len(cams), W, H))


def vrn_read_stats(ctx, workspace=None, stream=None) -> dict:
    lib = load_library()
    st = VrnStats()
    _check(lib.vrn_read_stats(ctx, _ptr(workspace), ctypes.byref(st), _stream(stream)), lib)
    return {name: int(getattr(st, name)) for name, _ in VrnStats._fields_}


def vrn_rays(ctx, cams, W, H, o, d, r, scale=1.0, stream=None):
    lib = load_library()
    arr = make_cameras(cams, H)
    _check(lib.vrn_rays(ctx, arr, len(cams), W, H, scale, _ptr(o), _ptr(d), _ptr(r), _stream(stream)),
           lib)


def vrn_march(ctx, fid, cams, W, H, klist, max_k, count, stream=None):
    lib = load_library()
    arr = make_cameras(cams, H)
    _check(lib.vrn_march(ctx, fid, arr, len(cams), W, H, _ptr(klist), max_k, _ptr(count),
                         _stream(stream)), lib)


def vrn_encode(ctx, fid, xyz, t, r, n, feat, stream=None):
    lib = load_library()
    _check(lib.vrn_encode(ctx, fid, _ptr(xyz), _ptr(t), _ptr(r), n, _ptr(feat), _stream(stream)), lib)


def vrn_mlp(ctx, fid, feat, dirs, n, compute, sigma, rgb, stream=None):
    lib = load_library()
    c = DTYPES[compute] if isinstance(compute, str) else int(compute)
    _check(lib.vrn_mlp(ctx, fid, _ptr(feat), _ptr(dirs), n, c, _ptr(sigma), _ptr(rgb),
                       _stream(stream)), lib)


def vrn_prune_grid(ctx, fid, alpha, bits_out, max_opacity=None, points_per_voxel=4, compute="f32",
                   stream=None):
    lib = load_library()
    c = DTYPES[compute] if isinstance(compute, str) else int(compute)
    _check(lib.vrn_prune_grid(ctx, fid, float(alpha), int(points_per_voxel), c, _ptr(bits_out),
                              _ptr(max_opacity), _stream(stream)), lib)


DEBUG_SLOTS = ("table_offset", "brick_index", "coarse_index", "pixel_write", "nan_feature", "nan_mlp_output")


def vrn_debug_counters(ctx, reset=False) -> dict:
    """Counters of a library built with -DVRN_DEBUG_CHECKS (raises
    VRN_ERR_UNSUPPORTED on a release build)."""
    lib = load_library()
    out = (c_u64 * len(DEBUG_SLOTS))()
    _check(lib.vrn_debug_counters(ctx, out, int(bool(reset))), lib)
    return dict(zip(DEBUG_SLOTS, (int(v) for v in out)))


PHASE_SLOTS = ("refill", "march", "encode", "mlp", "return", "composite")


def vrn_phase_cycles(ctx, reset=False) -> dict:
    """Shader clocks per step of the render waves' rounds, from a library
    built with -DVRN_PHASE_TIMING (raises VRN_ERR_UNSUPPORTED otherwise)."""
    lib = load_library()
    out = (c_u64 * len(PHASE_SLOTS))()
    _check(lib.vrn_phase_cycles(ctx, out, int(bool(reset))), lib)
    return dict(zip(PHASE_SLOTS, (int(v) for v in out)))


def vrn_set_occupancy(ctx, fid, bits, stream=None):
    lib = load_library()
    _check(lib.vrn_set_occupancy(ctx, fid, _ptr(bits), _stream(stream)), lib)


# ---------------------------------------------------------------------------
# serving engine
# ---------------------------------------------------------------------------

def vrn_server_create(ctx, arena_bytes, d_arena=None, n_slots=4, max_batch=4, use_graphs=True, compute="f16",
                      output=None, exposure_ev=0.0):
    """Create a serving engine (held: call vrn_server_hold(sv, False) to
    serve).  d_arena: a device tensor or address of >= arena_bytes, or None
    for an arena the engine allocates."""
    lib = load_library()
    o = VrnServerOpts()
    o.n_slots, o.max_batch, o.use_graphs = int(n_slots), int(max_batch), int(bool(use_graphs))
    o.render = render_opts(compute, output=output, exposure_ev=exposure_ev)
    o.d_arena = None if d_arena is None else _ptr(d_arena).value
    o.arena_bytes = int(arena_bytes)
    sv = c_vp()
    _check(lib.vrn_server_create(ctx, ctypes.byref(o), ctypes.byref(sv)), lib)
    return sv


def vrn_server_destroy(sv):
    load_library().vrn_server_destroy(sv)


def vrn_server_hold(sv, hold: bool):
    lib = load_library()
    _check(lib.vrn_server_hold(sv, int(bool(hold))), lib)


def vrn_server_prepare(sv, fid, n_cams, W, H):
    lib = load_library()
    _check(lib.vrn_server_prepare(sv, fid, n_cams, W, H), lib)


def vrn_server_submit(sv, fid, cams, W, H, t_arrival=0.0, timeout_s=0.0, flags=0, cam_array=None) -> int:
    """Queue a request; returns its id.  cam_array: the cameras already
    marshalled by make_cameras (skips the conversion)."""
    lib = load_library()
    arr = make_cameras(cams, H) if cam_array is None else cam_array
    ro = VrnRequestOpts(float(t_arrival), float(timeout_s), int(flags))
    rid = c_u64()
    _check(lib.vrn_server_submit(sv, fid, arr, len(arr), W, H, ctypes.byref(ro), ctypes.byref(rid)), lib)
    return int(rid.value)


def vrn_server_wait(sv, rid, max_wait_s=0.0):
    """(finished, VrnServed) for request rid after waiting up to max_wait_s."""
    lib = load_library()
    out = VrnServed()
    st = lib.vrn_server_wait(sv, rid, float(max_wait_s), ctypes.byref(out))
    if st == VRN_ERR_BUSY:
        return False, out
    _check(st, lib)
    return True, out


def vrn_server_release(sv, rid):
    lib = load_library()
    _check(lib.vrn_server_release(sv, rid), lib)


def vrn_server_cancel(sv, rid) -> bool:
    """True if the request was pending or running (it will finish cancelled);
    False if it had already finished."""
    lib = load_library()
    st = lib.vrn_server_cancel(sv, rid)
    if st == VRN_ERR_BUSY:
        return False
    _check(st, lib)
    return True


def vrn_server_drain(sv, max_wait_s=60.0):
    lib = load_library()
    _check(lib.vrn_server_drain(sv, float(max_wait_s)), lib)


def vrn_server_evict(sv, fid=0):
    lib = load_library()
    _check(lib.vrn_server_evict(sv, fid), lib)


def vrn_server_stats(sv) -> dict:
    lib = load_library()
    st = VrnServeStats()
    _check(lib.vrn_server_stats(sv, ctypes.byref(st)), lib)
    return {name: int(getattr(st, name)) for name, _ in VrnServeStats._fields_}


def vrn_server_clock() -> float:
    return float(load_library().vrn_server_clock())


# ---------------------------------------------------------------------------
# convenience
# ---------------------------------------------------------------------------

class Renderer:
    """One context on one device, with resident fields and a workspace."""

    def __init__(self, device: int = 0, hbm_budget_bytes: int = 0):
        import torch
        self.torch = torch
        self.device = torch.device("cuda", device)
        self.ctx = vrn_create(device, hbm_budget_bytes)
        self.ws = torch.zeros(vrn_workspace_bytes(self.ctx), dtype=torch.uint8, device=self.device)
        vrn_workspace_init(self.ctx, self.ws)

    def load(self, field) -> int:
        return vrn_load_field(self.ctx, field)

    def unload(self, fid):
        vrn_unload_field(self.ctx, fid)

    def render(self, fid, cams, W, H, compute="f32", linear_hdr=False, out=None, stream=None,
               march_budget=0, output=None, exposure_ev=0.0):
        torch = self.torch
        n = len(cams)
        if out is None:
            rgba = torch.zeros((n, H, W, 4), dtype=torch.float32, device=self.device)
            ns = torch.zeros((n, H, W), dtype=torch.int32, device=self.device)
        else:
            rgba, ns = out
        vrn_render(self.ctx, fid, cams, W, H, rgba, ns, compute, linear_hdr, self.ws, stream,
                   march_budget, output, exposure_ev)
        return rgba, ns

    def stats(self):
        return vrn_read_stats(self.ctx, self.ws)

    def close(self):
        if self.ctx is not None:
            vrn_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
