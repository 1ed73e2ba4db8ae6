"""Child process of tests/test_phase_timing.py: loads a libvrn built with
-DVRN_PHASE_TIMING, renders the stereo house frame (FP16 and FP32X) and the
unbounded scene (FP16), and prints each workload's shader clocks per step of
the waves' rounds as JSON."""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402
import torch  # noqa: E402

from paper_2311_02542_amd import capi, synth  # noqa: E402


def main(lib_path):
    torch.zeros(1, device="cuda")
    capi.load_library(lib_path)
    R = capi.Renderer(0)
    out = {}

    def run(name, field, cams_list, W, compute):
        fid = R.load(field)
        R.render(fid, cams_list[0], W, W, compute)
        torch.cuda.synchronize()
        capi.vrn_phase_cycles(R.ctx, reset=True)
        for cams in cams_list:
            R.render(fid, cams, W, W, compute)
        torch.cuda.synchronize()
        out[name] = capi.vrn_phase_cycles(R.ctx, reset=True)
        R.unload(fid)

    house32 = synth.field_house512(table_dtype=np.float32)
    house16 = dict(house32, tables=house32["tables"].astype(np.float16))
    frames = synth.cameras_house_stereo(range(0, 300, 60))
    run("house_f16", house16, frames, 2048, "f16")
    run("house_f32x", house32, frames[:2], 2048, "f32x")
    del house32, house16
    run("unbounded_f16", synth.field_unbounded(table_dtype=np.float16),
        [synth.cameras_unbounded(2, 2048, 2048)] * 3, 2048, "f16")
    R.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main(sys.argv[1])
