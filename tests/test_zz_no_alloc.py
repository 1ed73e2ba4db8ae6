"""The allocation-free render entry point (vrn_render_noalloc): its output
equals vrn_render_device_cams' bit for bit (same kernels, counters in the
library's static scratch instead of a workspace) on two calls in a row, the
second smaller than the first; graph replays of it equal eager calls; and
requests beyond its limits are refused on the host."""
import numpy as np
import pytest

from gpu_common import need_gpu
from paper_2311_02542_amd import capi, serve, synth

pytestmark = pytest.mark.gpu


def _dev_cams(torch, cams, H):
    blob = bytes(capi.make_cameras(cams, H))
    return torch.frombuffer(bytearray(blob), dtype=torch.uint8).cuda()


@pytest.mark.parametrize("compute", ["f32", "f16"])
def test_noalloc_equals_workspace_render_two_calls(compute):
    torch = need_gpu()
    R = capi.Renderer(0)
    fid = R.load(synth.field_blobs64())
    stream = torch.cuda.current_stream()
    ws = torch.zeros(capi.vrn_workspace_bytes(R.ctx), dtype=torch.uint8, device="cuda")
    capi.vrn_workspace_init(R.ctx, ws, stream=stream)
    # the second call is smaller than the first (fewer cameras, fewer pixels)
    for n_cams, W, H in ((2, 96, 80), (1, 40, 24)):
        cams = synth.cameras_blobs64(n_cams, W, H)
        dc = _dev_cams(torch, cams, H)
        a = torch.full((n_cams, H, W, 4), -1.0, device="cuda")
        an = torch.full((n_cams, H, W), -1, dtype=torch.int32, device="cuda")
        b = torch.full_like(a, -2.0)
        bn = torch.full_like(an, -2)
        capi.vrn_render_noalloc(R.ctx, fid, dc, n_cams, W, H, a, an, compute)
        capi.vrn_render_device_cams(R.ctx, fid, dc, n_cams, W, H, b, bn, compute, workspace=ws)
        torch.cuda.synchronize()
        assert torch.equal(a, b), f"{compute} {n_cams}x{W}x{H}: colors differ"
        assert torch.equal(an, bn), f"{compute} {n_cams}x{W}x{H}: sample counts differ"
        assert int(an.sum()) > 0 and bool((a[..., 3] >= 0).all())
    R.unload(fid)
    R.close()


def test_noalloc_graph_replays_equal_eager():
    torch = need_gpu()
    R = capi.Renderer(0)
    fid = R.load(synth.field_blobs64())
    W = H = 64
    cams_all = synth.cameras_blobs64(4, W, H)
    stream = torch.cuda.Stream()
    dcams = torch.zeros(serve.CAM_BYTES, dtype=torch.uint8, device="cuda")
    rgba = torch.zeros((1, H, W, 4), device="cuda")
    ns = torch.zeros((1, H, W), dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=stream, capture_error_mode="thread_local"):
        capi.vrn_render_noalloc(R.ctx, fid, dcams, 1, W, H, rgba, ns, "f16", stream=stream)
    for rep in range(4):
        dcams.copy_(_dev_cams(torch, [cams_all[rep]], H))
        torch.cuda.synchronize()
        with torch.cuda.stream(stream):
            g.replay()
        stream.synchronize()
        got, got_n = rgba.clone(), ns.clone()
        # eager work between replays: the same camera through the eager entry point
        ref = torch.zeros_like(rgba)
        ref_n = torch.zeros_like(ns)
        capi.vrn_render_noalloc(R.ctx, fid, dcams, 1, W, H, ref, ref_n, "f16")
        torch.cuda.synchronize()
        assert torch.equal(got, ref) and torch.equal(got_n, ref_n), f"replay {rep}"
    R.unload(fid)
    R.close()


def test_noalloc_refuses_requests_beyond_its_limits():
    torch = need_gpu()
    R = capi.Renderer(0)
    fid = R.load(synth.field_blobs64())
    dc = torch.zeros(serve.CAM_BYTES * (capi.MAX_CAMS + 1), dtype=torch.uint8, device="cuda")
    rgba = torch.zeros(16, device="cuda")
    for n_cams, W, H in ((capi.MAX_CAMS + 1, 8, 8), (1, 16385, 8), (1, 8, 0), (16, 16384, 16384)):
        with pytest.raises(capi.VrnError) as ei:
            capi.vrn_render_noalloc(R.ctx, fid, dc, n_cams, W, H, rgba)
        assert ei.value.status == capi.VRN_ERR_INVALID_ARG
    with pytest.raises(capi.VrnError) as ei:
        capi.vrn_render_noalloc(R.ctx, 999, dc, 1, 8, 8, rgba)
    assert ei.value.status == capi.VRN_ERR_NOT_FOUND
    R.unload(fid)
    R.close()
