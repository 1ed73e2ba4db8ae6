"""Device-side checks of a debug build (-DVRN_DEBUG_CHECKS): the kernels
count, rather than trap on, hash-table offsets outside their level, brick
and coarse-grid indices outside the grid, framebuffer writes outside the
frame and NaN features or MLP outputs.  Every workload kind (the stereo
house frame in FP16, BF16, FP32 and FP32X; the unbounded scene; the exponential
sample table; the room; grid pruning; the encode and MLP stage kernels) runs
through a debug build in a child process and must leave every counter at
zero, while an FP16 field whose weights overflow must be counted (the
positive control of the NaN counter)."""
import json
import os
import subprocess
import sys

import pytest

from paper_2311_02542_amd import capi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2311_02542_amd", "csrc")
from paper_2311_02542_amd.build import SOURCES  # noqa: E402
HIPCC = "/opt/rocm/bin/hipcc"


def test_debug_counters_argument_check():
    lib = capi.load_library()
    assert lib.vrn_debug_counters(None, None, 0) == capi.VRN_ERR_INVALID_ARG


@pytest.mark.gpu
def test_release_build_reports_unsupported():
    from gpu_common import need_gpu
    need_gpu()
    R = capi.Renderer(0)
    try:
        with pytest.raises(capi.VrnError) as ei:
            capi.vrn_debug_counters(R.ctx)
        assert ei.value.status == capi.VRN_ERR_UNSUPPORTED
    finally:
        R.close()


@pytest.mark.gpu
def test_debug_build_counts_no_violations(tmp_path):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    lib = str(tmp_path / "libvrn_debug.so")
    flags = ("--offload-arch=gfx950 -O3 -std=c++17 -fPIC -shared -ffp-contract=off "
             "-fhip-fp32-correctly-rounded-divide-sqrt -Xclang -target-feature -Xclang -packed-fp32-ops "
             "-Wno-unused-result -Wno-unused-value -DVRN_DEBUG_CHECKS").split()
    res = subprocess.run([HIPCC, *flags, "-I", os.path.join(ROOT, "include"), "-I", CSRC,
                          *SOURCES, "-o", lib],
                         capture_output=True, text=True)
    assert res.returncode == 0, res.stderr[-3000:]
    res = subprocess.run([sys.executable, os.path.join(ROOT, "tests", "debug_checks_driver.py"), lib],
                         capture_output=True, text=True, timeout=300)
    print(res.stdout, res.stderr[-3000:])
    assert res.returncode == 0, res.stderr[-3000:]
    out = json.loads(res.stdout.strip().splitlines()[-1])
    assert out["rays"] > 8_000_000
    assert all(v == 0 for v in out["counts"].values()), out["counts"]
    assert out["control"]["nan_mlp_output"] > 0, out["control"]
