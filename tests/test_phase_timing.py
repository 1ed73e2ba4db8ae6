"""The phase-timing build (-DVRN_PHASE_TIMING): render waves sum the shader
clocks of each step of their rounds (refill, march, encode, MLP, return of
the results, compositing), read through vrn_phase_cycles.  Release builds
compile none of it and report VRN_ERR_UNSUPPORTED.  On the GPU the build's
profile must show every step of a render, and the march must take a larger
share of the waves' time on the unbounded scene (31.5 lattice tests per ray
for 1.7 samples) than on the house frame (20.5 for 5.0)."""
import json
import os
import subprocess
import sys

import pytest

from paper_2311_02542_amd import capi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2311_02542_amd", "csrc")
from paper_2311_02542_amd.build import FLAGS, SOURCES, hipcc  # noqa: E402


def test_phase_cycles_argument_check():
    lib = capi.load_library()
    assert lib.vrn_phase_cycles(None, None, 0) == capi.VRN_ERR_INVALID_ARG


@pytest.mark.gpu
def test_release_build_reports_unsupported():
    from gpu_common import need_gpu
    need_gpu()
    R = capi.Renderer(0)
    try:
        with pytest.raises(capi.VrnError) as ei:
            capi.vrn_phase_cycles(R.ctx)
        assert ei.value.status == capi.VRN_ERR_UNSUPPORTED
    finally:
        R.close()


@pytest.mark.gpu
def test_phase_timing_build_profiles_every_step(tmp_path):
    lib = str(tmp_path / "libvrn_phase.so")
    res = subprocess.run([hipcc(), *FLAGS, "-DVRN_PHASE_TIMING", "-I", os.path.join(ROOT, "include"), "-I", CSRC,
                          *SOURCES, "-o", lib], capture_output=True, text=True)
    assert res.returncode == 0, res.stderr[-3000:]
    res = subprocess.run([sys.executable, os.path.join(ROOT, "tests", "phase_timing_driver.py"), lib],
                         capture_output=True, text=True, timeout=300)
    print(res.stdout, res.stderr[-3000:])
    assert res.returncode == 0, res.stderr[-3000:]
    out = json.loads(res.stdout.strip().splitlines()[-1])
    share = {}
    for name, ph in out.items():
        total = sum(ph.values())
        assert total > 0
        share[name] = {k: v / total for k, v in ph.items()}
        print(name, {k: round(v, 3) for k, v in share[name].items()})
        for step in ("refill", "march", "encode", "mlp", "return", "composite"):
            assert ph[step] > 0, (name, step)
    assert share["unbounded_f16"]["march"] > share["house_f16"]["march"] + 0.2
    # the house frame's waves spend most of their time gathering and encoding
    assert share["house_f16"]["encode"] > share["house_f16"]["mlp"]
