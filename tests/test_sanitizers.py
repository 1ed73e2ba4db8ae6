"""Host code of the C ABI under AddressSanitizer and UndefinedBehaviorSanitizer.

libvrn is rebuilt with the sanitizers on its host code only (each
-fsanitize= behind -Xarch_host; the gfx950 device code is built as usual),
and two plain C clients built with clang's sanitizer runtime call it:
tests/c_abi_validation.c drives every host-side argument check at the edges
of its ranges without a GPU, and tests/c_abi_render.c (on the GPU) loads a
field, renders it and checks the compositing closed form, which runs the
host code of field loading (validation, occupancy bricks and coarse grids,
MFMA weight layout), rendering and unloading under the sanitizers.  Any
sanitizer report aborts the client with a non-zero status."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2311_02542_amd", "csrc")
from paper_2311_02542_amd.build import SOURCES  # noqa: E402
ROCM = "/opt/rocm"
HIPCC = os.path.join(ROCM, "bin", "hipcc")
CLANG = os.path.join(ROCM, "llvm", "bin", "clang")
DEVICE_FLAGS = ("--offload-arch=gfx950 -O1 -g -std=c++17 -fPIC -shared -ffp-contract=off "
                "-fhip-fp32-correctly-rounded-divide-sqrt -Xclang -target-feature -Xclang -packed-fp32-ops "
                "-Wno-unused-result -Wno-unused-value").split()
HOST_SANITIZERS = ("-Xarch_host -fsanitize=address -Xarch_host -fsanitize=undefined "
                   "-Xarch_host -fno-sanitize-recover=undefined -Xarch_host -fno-omit-frame-pointer").split()
CLIENT_SANITIZERS = "-fsanitize=address,undefined -fno-sanitize-recover=undefined -fno-omit-frame-pointer".split()


@pytest.fixture(scope="module")
def sanitized_lib(tmp_path_factory):
    if not (os.path.exists(HIPCC) and os.path.exists(CLANG)):
        pytest.skip("hipcc / clang not available")
    out = tmp_path_factory.mktemp("san")
    lib = str(out / "libvrn_san.so")
    cmd = [HIPCC, *DEVICE_FLAGS, *HOST_SANITIZERS, "-I", os.path.join(ROOT, "include"), "-I", CSRC,
           *SOURCES, "-o", lib]
    res = subprocess.run(cmd, capture_output=True, text=True)
    assert res.returncode == 0, res.stderr[-3000:]
    return out


def _client(out, name, gpu):
    exe = str(out / name)
    cmd = [CLANG, "-std=c11", "-g", "-O1", "-Wall", "-Wextra", "-Werror", *CLIENT_SANITIZERS,
           "-I", os.path.join(ROOT, "include"), os.path.join(ROOT, "tests", name + ".c"), "-o", exe,
           "-L", str(out), "-l:libvrn_san.so", f"-Wl,-rpath,{out}", f"-Wl,-rpath,{os.path.join(ROCM, 'lib')}", "-lm"]
    if gpu:
        cmd[1:1] = ["-D__HIP_PLATFORM_AMD__", "-isystem", os.path.join(ROCM, "include")]
        cmd += ["-L", os.path.join(ROCM, "lib"), "-lamdhip64"]
    res = subprocess.run(cmd, capture_output=True, text=True)
    assert res.returncode == 0, res.stderr[-3000:]
    return exe


def _run(exe, detect_leaks):
    env = dict(os.environ, ASAN_OPTIONS=f"detect_leaks={int(detect_leaks)}:abort_on_error=0")
    res = subprocess.run([exe], capture_output=True, text=True, timeout=120, env=env)
    print(res.stdout, res.stderr[-3000:])
    return res


def test_host_validation_is_sanitizer_clean(sanitized_lib):
    """Every host-side check, driven from C at the edges of its ranges: the
    expected status each time, no ASan, UBSan or leak report."""
    res = _run(_client(sanitized_lib, "c_abi_validation", gpu=False), detect_leaks=True)
    assert res.returncode == 0, res.stderr[-3000:]


@pytest.mark.gpu
def test_load_render_unload_is_sanitizer_clean(sanitized_lib):
    """A field load, a render checked against the compositing closed form and
    an unload, with the library's host code under ASan and UBSan (leak
    checking off: the HIP runtime keeps process-lifetime allocations)."""
    res = _run(_client(sanitized_lib, "c_abi_render", gpu=True), detect_leaks=False)
    assert res.returncode == 0, res.stderr[-3000:]
