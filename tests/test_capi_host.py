"""Host-side tests of the C ABI: the library builds, loads and exports every
symbol include/vrn.h declares; argument validation runs on the host before
any device work (so these paths are testable without a GPU)."""
import ctypes
import math
import os

import numpy as np
import pytest

from paper_2311_02542_amd import capi, synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(capi.LIB_PATH):
        from paper_2311_02542_amd import build
        build.build()
    return capi.load_library()


def test_exports_every_header_symbol(lib):
    names = capi.header_symbols()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), n


def test_create_without_device_reports_device_error(lib):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    ctx = ctypes.c_void_p()
    assert lib.vrn_create(0, 0, ctypes.byref(ctx)) == capi.VRN_ERR_DEVICE
    assert "device" in lib.vrn_last_error().decode()
    assert lib.vrn_create(0, 0, None) == capi.VRN_ERR_INVALID_ARG


def _cam(**kw):
    c = synth.cameras_blobs64(1)[0]
    c = dict(c)
    c.update(kw)
    return c


def test_camera_validation(lib):
    assert capi.vrn_check_cameras([_cam()], 64, 64) == capi.VRN_OK
    bad = _cam()
    bad["c2w"] = bad["c2w"].copy()
    bad["c2w"][0, 0] = np.nan
    assert capi.vrn_check_cameras([bad], 64, 64) == capi.VRN_ERR_INVALID_ARG
    deg = _cam()
    deg["c2w"] = deg["c2w"].copy()
    deg["c2w"][:, 1] = deg["c2w"][:, 0]          # degenerate rotation
    assert capi.vrn_check_cameras([deg], 64, 64) == capi.VRN_ERR_INVALID_ARG
    assert capi.vrn_check_cameras([_cam(fx=np.float32(0))], 64, 64) == capi.VRN_ERR_INVALID_ARG
    assert capi.vrn_check_cameras([_cam(row_begin=10, row_end=10)], 64, 64) == capi.VRN_ERR_INVALID_ARG
    assert capi.vrn_check_cameras([_cam(row_begin=0, row_end=65)], 64, 64) == capi.VRN_ERR_INVALID_ARG
    assert capi.vrn_check_cameras([_cam()], 0, 64) == capi.VRN_ERR_INVALID_ARG
    assert capi.vrn_check_cameras([_cam()] * 17, 64, 64) == capi.VRN_ERR_INVALID_ARG


def test_render_rejects_bad_cameras_before_device_work(lib):
    bad = _cam()
    bad["c2w"] = bad["c2w"].copy()
    bad["c2w"][1, 3] = np.inf
    arr = capi.make_cameras([bad], 64)
    st = lib.vrn_render(None, 1, arr, 1, 64, 64, None, None, None, None, 0, None)
    assert st == capi.VRN_ERR_INVALID_ARG
    arr = capi.make_cameras([_cam()], 64)
    st = lib.vrn_render(None, 1, arr, 1, 64, 64, None, None, None, None, 0, None)
    assert st == capi.VRN_ERR_INVALID_ARG      # NULL context


def _desc_status(lib, field, **over):
    d, keep = capi.make_field_desc(field)
    for k, v in over.items():
        setattr(d, k, v)
    fid = ctypes.c_uint32()
    return lib.vrn_load_field(None, ctypes.byref(d), ctypes.byref(fid))


def test_field_validation(lib):
    f = synth.field_blobs64()
    assert _desc_status(lib, f) == capi.VRN_ERR_INVALID_ARG          # valid field, NULL ctx
    assert _desc_status(lib, f, n_feat=4) == capi.VRN_ERR_UNSUPPORTED
    assert _desc_status(lib, f, n_levels=17) == capi.VRN_ERR_UNSUPPORTED
    assert _desc_status(lib, f, log2_T=30) == capi.VRN_ERR_UNSUPPORTED
    assert _desc_status(lib, f, mlp_hidden=128) == capi.VRN_ERR_UNSUPPORTED
    assert _desc_status(lib, f, sh_bands=5) == capi.VRN_ERR_UNSUPPORTED
    assert _desc_status(lib, f, occ_res=2048) == capi.VRN_ERR_UNSUPPORTED
    assert _desc_status(lib, f, mlp_in=15) == capi.VRN_ERR_INVALID_ARG
    assert _desc_status(lib, f, dt=0.0) == capi.VRN_ERR_INVALID_ARG
    assert _desc_status(lib, f, extent=float("nan")) == capi.VRN_ERR_INVALID_ARG
    assert _desc_status(lib, f, t_min=1.0) == capi.VRN_ERR_INVALID_ARG
    assert _desc_status(lib, f, max_samples=0) == capi.VRN_ERR_INVALID_ARG
    assert _desc_status(lib, f, lod_enable=1, growth=1.0) == capi.VRN_ERR_INVALID_ARG
    assert _desc_status(lib, f, table_dtype=2) == capi.VRN_ERR_UNSUPPORTED
    assert "table_dtype" in lib.vrn_last_error().decode()


@pytest.mark.parametrize("over,status,words", [
    (dict(n_levels=0), capi.VRN_ERR_UNSUPPORTED, "n_levels"),
    (dict(log2_T=3), capi.VRN_ERR_UNSUPPORTED, "log2_T"),
    (dict(occ_res=0), capi.VRN_ERR_UNSUPPORTED, "occ_res"),
    (dict(sh_bands=0), capi.VRN_ERR_UNSUPPORTED, "sh_bands"),
    (dict(geo_out=8), capi.VRN_ERR_UNSUPPORTED, "geo_out"),
    (dict(tables=None), capi.VRN_ERR_INVALID_ARG, "NULL"),
    (dict(weights=None), capi.VRN_ERR_INVALID_ARG, "NULL"),
    (dict(occ_bits=None), capi.VRN_ERR_INVALID_ARG, "NULL"),
    (dict(level_res=None), capi.VRN_ERR_INVALID_ARG, "NULL"),
    (dict(t_min=-1e-4), capi.VRN_ERR_INVALID_ARG, "t_min"),
    (dict(extent=-1.0), capi.VRN_ERR_INVALID_ARG, "extent"),
    (dict(dt=float("inf")), capi.VRN_ERR_INVALID_ARG, "dt"),
    (dict(contraction=2), capi.VRN_ERR_INVALID_ARG, "contraction"),
    (dict(contraction=1), capi.VRN_ERR_INVALID_ARG, "aabb_min = -2"),
    (dict(step_growth=1.0), capi.VRN_ERR_INVALID_ARG, "step_growth"),
    (dict(step_growth=-0.5), capi.VRN_ERR_INVALID_ARG, "step_growth"),
    (dict(step_growth=0.01, max_lattice=0), capi.VRN_ERR_INVALID_ARG, "max_lattice"),
    (dict(step_growth=0.01, max_lattice=70000), capi.VRN_ERR_INVALID_ARG, "max_lattice"),
    (dict(lod_enable=1, base_res=0.0), capi.VRN_ERR_INVALID_ARG, "base_res"),
    (dict(lod_enable=1, lod_bias=float("nan")), capi.VRN_ERR_INVALID_ARG, "lod_bias"),
    (dict(lod_enable=1, lod_radius_scale=0.0), capi.VRN_ERR_INVALID_ARG, "lod_radius_scale"),
])
def test_field_validation_more(lib, over, status, words):
    """Every descriptor check runs on the host before the context is touched
    (a NULL context here), with its own status and message."""
    assert _desc_status(lib, synth.field_blobs64(), **over) == status
    assert words in lib.vrn_last_error().decode()


def test_contracted_field_geometry_checks(lib):
    f = synth.field_unbounded()
    assert _desc_status(lib, f) == capi.VRN_ERR_INVALID_ARG                  # valid; NULL ctx
    assert "ctx" in lib.vrn_last_error().decode()
    assert _desc_status(lib, f, extent=8.0) == capi.VRN_ERR_INVALID_ARG
    assert "extent = 4" in lib.vrn_last_error().decode()
    assert _desc_status(lib, f, radius=0.0) == capi.VRN_ERR_INVALID_ARG
    assert "radius" in lib.vrn_last_error().decode()


def test_level_resolution_bounds(lib):
    f = synth.field_blobs64()
    for bad in (0, (1 << 20) + 1):
        res = np.array(f["level_res"], np.uint32)
        res[-1] = bad
        assert _desc_status(lib, dict(f, level_res=res)) == capi.VRN_ERR_INVALID_ARG
        assert "level_res" in lib.vrn_last_error().decode()


def test_field_file_round_trip_two_readers(tmp_path):
    """The writer's files are read back identically by the oracle's reader and
    by the product binding's descriptor marshalling."""
    from oracle.field_io import load_field
    f = synth.field_blobs64()
    prefix = str(tmp_path / "blobs64")
    synth.save_field(prefix, f)
    g = load_field(prefix)
    for k in ("level_res", "hash_primes", "tables", "occ_bits", "aabb_min"):
        assert np.array_equal(np.asarray(g[k]), np.asarray(f[k])), k
    for k in f["mlp"]:
        assert np.array_equal(g["mlp"][k], f["mlp"][k])
    for k in ("n_levels", "log2_T", "occ_res", "max_samples", "sh_bands", "lod_enable"):
        assert g[k] == f[k]
    for k in ("extent", "dt", "t_min", "base_res", "growth"):
        assert np.float32(g[k]) == np.float32(f[k])
    d1, _ = capi.make_field_desc(f)
    d2, _ = capi.make_field_desc(g)
    for name, t in capi.VrnFieldDesc._fields_:
        if t in (capi.c_u32, capi.c_i32, capi.c_f):
            assert getattr(d1, name) == getattr(d2, name), name


def test_server_entry_points_validate_on_host(lib):
    """The serving engine's entry points refuse NULL handles and options out
    of range before touching a context or the device."""
    P = ctypes.byref
    out = ctypes.c_void_p()
    opts = capi.VrnServerOpts()
    opts.n_slots, opts.max_batch, opts.use_graphs, opts.arena_bytes = 2, 4, 1, 1 << 20
    opts.render = capi.render_opts("f16")
    assert lib.vrn_server_create(None, P(opts), P(out)) == capi.VRN_ERR_INVALID_ARG
    # a stand-in context handle: every case below is refused before it is read
    dummy = ctypes.create_string_buffer(64)
    ctx = ctypes.c_void_p(ctypes.addressof(dummy))
    assert lib.vrn_server_create(ctx, None, P(out)) == capi.VRN_ERR_INVALID_ARG
    bad = [("n_slots", 0), ("n_slots", 17), ("max_batch", 0), ("max_batch", capi.MAX_CAMS + 1),
           ("use_graphs", 2), ("arena_bytes", 255)]
    for name, v in bad:
        o = capi.VrnServerOpts.from_buffer_copy(opts)
        setattr(o, name, v)
        assert lib.vrn_server_create(ctx, P(o), P(out)) == capi.VRN_ERR_INVALID_ARG, name
        assert out.value is None
    o = capi.VrnServerOpts.from_buffer_copy(opts)
    o.render.compute = 7
    assert lib.vrn_server_create(ctx, P(o), P(out)) == capi.VRN_ERR_INVALID_ARG
    o = capi.VrnServerOpts.from_buffer_copy(opts)
    o.render.exposure_ev = math.inf
    assert lib.vrn_server_create(ctx, P(o), P(out)) == capi.VRN_ERR_INVALID_ARG
    o = capi.VrnServerOpts.from_buffer_copy(opts)
    o.d_arena = 0x1000 + 16                     # not 256-byte aligned
    assert lib.vrn_server_create(ctx, P(o), P(out)) == capi.VRN_ERR_INVALID_ARG
    assert "aligned" in lib.vrn_last_error().decode()
    # NULL engine handle
    rid = ctypes.c_uint64()
    served = capi.VrnServed()
    st = capi.VrnServeStats()
    arr = capi.make_cameras([_cam()], 64)
    assert lib.vrn_server_submit(None, 1, arr, 1, 64, 64, None, P(rid)) == capi.VRN_ERR_INVALID_ARG
    assert lib.vrn_server_wait(None, 1, 0.0, P(served)) == capi.VRN_ERR_INVALID_ARG
    assert lib.vrn_server_hold(None, 1) == capi.VRN_ERR_INVALID_ARG
    assert lib.vrn_server_prepare(None, 1, 1, 64, 64) == capi.VRN_ERR_INVALID_ARG
    assert lib.vrn_server_release(None, 1) == capi.VRN_ERR_INVALID_ARG
    assert lib.vrn_server_cancel(None, 1) == capi.VRN_ERR_INVALID_ARG
    assert lib.vrn_server_drain(None, 0.0) == capi.VRN_ERR_INVALID_ARG
    assert lib.vrn_server_evict(None, 0) == capi.VRN_ERR_INVALID_ARG
    assert lib.vrn_server_stats(None, P(st)) == capi.VRN_ERR_INVALID_ARG
    lib.vrn_server_destroy(None)                # a no-op


def test_server_clock_is_monotonic_seconds(lib):
    import time
    a = capi.vrn_server_clock()
    m = time.monotonic()
    time.sleep(0.01)
    b = capi.vrn_server_clock()
    assert 0.009 < b - a < 1.0
    assert abs(a - m) < 1.0                     # CLOCK_MONOTONIC, as time.monotonic
