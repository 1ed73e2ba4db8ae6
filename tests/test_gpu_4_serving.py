"""Serving systems tests: HIP graph replay equals eager launches (several
replays with eager work and synchronisation in between), a request gives the
same result alone and inside a concurrent mix (bitwise: every ray's
arithmetic is independent of batch composition), HBM-budget admission and
queueing, and unload of a busy field."""
import time

import numpy as np
import pytest

from gpu_common import need_gpu
from paper_2311_02542_amd import capi, serve, synth

pytestmark = pytest.mark.gpu


def test_graph_replay_equals_eager():
    torch = need_gpu()
    R = capi.Renderer(0)
    f = synth.field_blobs64()
    fid = R.load(f)
    W = H = 96
    cams_all = synth.cameras_blobs64(5, W, H)
    stream = torch.cuda.Stream()
    ws = torch.zeros(capi.vrn_workspace_bytes(R.ctx), dtype=torch.uint8, device="cuda")
    capi.vrn_workspace_init(R.ctx, ws, stream=stream)
    dcams = torch.zeros(serve.CAM_BYTES * 2, dtype=torch.uint8, device="cuda")
    rgba = torch.zeros((2, H, W, 4), device="cuda")
    ns = torch.zeros((2, H, W), dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=stream, capture_error_mode="thread_local"):
        capi.vrn_render_device_cams(R.ctx, fid, dcams, 2, W, H, rgba, ns, "f16", workspace=ws, stream=stream)
    for rep in range(4):
        pair = [cams_all[rep], cams_all[rep + 1]]
        blob = bytes(capi.make_cameras(pair, H))
        dcams.copy_(torch.frombuffer(bytearray(blob), dtype=torch.uint8).cuda())
        torch.cuda.synchronize()
        with torch.cuda.stream(stream):
            g.replay()
        stream.synchronize()
        got_rgba, got_ns = rgba.clone(), ns.clone()
        # eager work between replays
        ref_rgba, ref_ns = R.render(fid, pair, W, H, "f16")
        torch.cuda.synchronize()
        assert torch.equal(got_rgba, ref_rgba) and torch.equal(got_ns, ref_ns), f"replay {rep}"
    R.unload(fid)
    R.close()


def _fields():
    return {"A": synth.field_blobs64(), "B": synth.field_blobs_3m2()}


def test_alone_vs_mix_bitwise():
    torch = need_gpu()
    srv = serve.Server(_fields(), 4 << 30, n_slots=3, compute="f16", use_graphs=True)
    probe = synth.request_cameras("A", "tile", 1234)
    srv.start()
    alone = srv.submit("A", *probe)
    alone.done.wait(30)
    srv.stop()
    # a mixed burst around the same request (batched with other same-size tiles)
    srv.start()
    mix = []
    rng = np.random.default_rng(0)
    for i in range(24):
        scene = "AB"[i % 2]
        kind = ["preview", "tile", "stereo"][rng.integers(3)]
        cams, W, H = synth.request_cameras(scene, kind, int(rng.integers(1 << 30)))
        mix.append(srv.submit(scene, cams, W, H))
        if i == 9:
            target = srv.submit("A", *probe)
    srv.stop(drain=True)
    torch.cuda.synchronize()
    assert all(r.done.is_set() for r in mix) and target.done.is_set()
    assert torch.equal(alone.result[0], target.result[0])
    assert torch.equal(alone.result[1], target.result[1])
    # spot-check a mixed request against a direct render
    R = capi.Renderer(0)
    r = mix[5]
    fid = R.load(_fields()[r.scene])
    ref, _ = R.render(fid, r.cams, r.W, r.H, "f16")
    torch.cuda.synchronize()
    assert torch.equal(ref, r.result[0])
    R.unload(fid)
    R.close()
    srv.close()


def test_admission_budget_and_queueing():
    torch = need_gpu()
    fields = {"A": synth.field_blobs64()}
    fbytes = synth.field_bytes(fields["A"])
    # budget fits the field, the slot workspaces and ONE 1024^2 output buffer at a time
    budget = fbytes * 2 + (1 << 20) + 1024 * 1024 * 20 + (1 << 20)
    srv = serve.Server(fields, budget, n_slots=2, compute="f16", use_graphs=False)
    with pytest.raises(serve.ServeError):
        srv.submit("A", *synth.request_cameras("A", "stereo", 1))     # 2x2048^2 can never fit
    srv.start()
    reqs = [srv.submit("A", *synth.request_cameras("A", "tile", 100 + i)) for i in range(4)]
    srv.stop(drain=True)
    assert all(r.done.is_set() for r in reqs)
    R = capi.Renderer(0)
    fid = R.load(fields["A"])
    for r in reqs:
        ref, _ = R.render(fid, r.cams, r.W, r.H, "f16")
        torch.cuda.synchronize()
        assert torch.equal(ref, r.result[0])
    R.unload(fid)
    R.close()
    srv.close()
    # a context budget below the field size refuses the load
    ctx = capi.vrn_create(0, fbytes // 2)
    with pytest.raises(capi.VrnError) as ei:
        capi.vrn_load_field(ctx, fields["A"])
    assert ei.value.status == capi.VRN_ERR_BUDGET
    capi.vrn_destroy(ctx)


def test_drain_waits_for_a_batch_being_launched():
    """stop(drain=True) must not return while the loop holds a batch it has
    taken from the queue but not yet put on a slot: _launch is slowed down
    here so that a drain check always falls into that window."""
    need_gpu()
    srv = serve.Server({"A": synth.field_blobs64()}, 8 << 30, n_slots=1, compute="f16", use_graphs=False)
    launch = srv._launch

    def slow_launch(slot, reqs):
        time.sleep(0.05)
        return launch(slot, reqs)

    srv._launch = slow_launch
    srv.start()
    reqs = [srv.submit("A", *synth.request_cameras("A", "preview", 7 + i)) for i in range(3)]
    srv.stop(drain=True)
    try:
        assert all(r.done.is_set() and r.error is None for r in reqs)
    finally:
        srv.close()


def test_unload_busy_field_and_errors():
    torch = need_gpu()
    R = capi.Renderer(0)
    f = synth.field_house512(table_dtype=np.float16)
    fid = R.load(f)
    cams = synth.cameras_house_stereo([0])[0]
    rgba = torch.zeros((2, 2048, 2048, 4), device="cuda")
    capi.vrn_render(R.ctx, fid, cams, 2048, 2048, rgba, None, "f32", workspace=R.ws)
    with pytest.raises(capi.VrnError) as ei:
        capi.vrn_unload_field(R.ctx, fid)
    assert ei.value.status == capi.VRN_ERR_BUSY
    torch.cuda.synchronize()
    capi.vrn_unload_field(R.ctx, fid)
    with pytest.raises(capi.VrnError) as ei:
        capi.vrn_unload_field(R.ctx, fid)
    assert ei.value.status == capi.VRN_ERR_NOT_FOUND
    with pytest.raises(capi.VrnError) as ei:
        capi.vrn_render(R.ctx, 999, cams, 2048, 2048, rgba, None)
    assert ei.value.status == capi.VRN_ERR_NOT_FOUND
    R.close()


def test_warmup_captures_buckets_and_serves_exactly():
    """Graphs captured ahead of serving (every slot, scene and shape) replay
    requests bit-for-bit like a direct render, with no new bucket created."""
    torch = need_gpu()
    srv = serve.Server(_fields(), 4 << 30, n_slots=2, compute="f16", use_graphs=True)
    shapes = [(256, 256, 1), (256, 256, 2)]
    srv.warmup(shapes)
    keys = {k for s in srv.slots for k in s.buckets}
    assert keys == {(sc, w, h, n, "f16") for sc in ("A", "B") for (w, h, n) in shapes}
    srv.start()
    reqs = [srv.submit(sc, *synth.request_cameras(sc, "preview", 50 + i)) for i, sc in enumerate("ABAB")]
    srv.stop(drain=True)
    assert {k for s in srv.slots for k in s.buckets} == keys
    R = capi.Renderer(0)
    fids = {name: R.load(f) for name, f in _fields().items()}
    for r in reqs:
        assert r.error is None and r.done.is_set()
        ref, ref_n = R.render(fids[r.scene], r.cams, r.W, r.H, "f16")
        torch.cuda.synchronize()
        assert torch.equal(ref, r.result[0]) and torch.equal(ref_n, r.result[1])
    for fid in fids.values():
        R.unload(fid)
    R.close()
    srv.close()
