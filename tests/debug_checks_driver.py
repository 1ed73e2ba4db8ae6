"""Child process of tests/test_debug_checks.py: loads a libvrn built with
-DVRN_DEBUG_CHECKS, runs every kind of workload through it and prints the
debug counters as JSON.  A field whose density weights overflow FP16 is
rendered last on the FP16 path, as a positive control of the NaN counter."""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402
import torch  # noqa: E402

from paper_2311_02542_amd import capi, synth  # noqa: E402


def main(lib_path):
    capi.load_library(lib_path)
    R = capi.Renderer(0)
    rays = 0

    def render(field, cams, W, H, paths):
        nonlocal rays
        fid = R.load(field)
        for p in paths:
            R.render(fid, cams, W, H, p)
            rays += len(cams) * W * H
        torch.cuda.synchronize()
        R.unload(fid)

    house32 = synth.field_house512(table_dtype=np.float32)
    house16 = dict(house32, tables=house32["tables"].astype(np.float16))
    stereo = synth.cameras_house_stereo([150])[0]
    render(house16, stereo, 2048, 2048, ["f16", "bf16"])
    render(house32, stereo, 2048, 2048, ["f32", "f32x"])
    del house32, house16
    render(synth.field_unbounded(), synth.cameras_unbounded(2, 256, 256), 256, 256, ["f32"])
    render(synth.field_unbounded(table_dtype=np.float16), synth.cameras_unbounded(2, 256, 256), 256, 256, ["f16"])
    expo = dict(synth.field_blobs64(), step_growth=float(np.float32(1 / 32)), max_lattice=300)
    render(expo, synth.cameras_blobs64(3), 64, 64, ["f32", "f16"])
    render(synth.field_room256(), synth.cameras_room256(1, 512, 512), 512, 512, ["f32"])
    # pruning and the stage kernels
    blob = synth.field_blobs64()
    fid = R.load(blob)
    bits = torch.zeros(((64 ** 3 + 31) // 32,), dtype=torch.int32, device="cuda")
    for p in ("f16", "f32", "f32x"):
        capi.vrn_prune_grid(R.ctx, fid, 0.2, bits, None, 4, p)
    n = 4096
    g = torch.Generator().manual_seed(3)
    xyz = (torch.rand((n, 3), generator=g) * 1.2 - 0.1).cuda()
    feat = torch.zeros((n, 2 * int(blob["n_levels"])), device="cuda")
    capi.vrn_encode(R.ctx, fid, xyz, None, None, n, feat)
    dirs = torch.nn.functional.normalize(torch.randn((n, 3), generator=g), dim=1).cuda()
    sigma, rgb = torch.zeros(n, device="cuda"), torch.zeros((n, 3), device="cuda")
    capi.vrn_mlp(R.ctx, fid, feat, dirs, n, "f16", sigma, rgb)
    torch.cuda.synchronize()
    R.unload(fid)
    counts = capi.vrn_debug_counters(R.ctx, reset=True)
    # positive control: one feature's first-layer weights of 1e6 are finite but
    # overflow FP16, so samples with that feature positive get +inf hidden units,
    # which the next layer's mixed-sign weights turn into NaN outputs
    hot = synth.field_blobs64()
    hot["mlp"] = {k: v.copy() for k, v in hot["mlp"].items()}
    hot["mlp"]["W1"][0, :] = 1.0e6
    render(hot, synth.cameras_blobs64(1, 32, 32), 32, 32, ["f16"])
    control = capi.vrn_debug_counters(R.ctx, reset=True)
    R.close()
    print(json.dumps({"rays": rays, "counts": counts, "control": control}), flush=True)


if __name__ == "__main__":
    main(sys.argv[1])
