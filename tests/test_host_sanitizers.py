"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

scene.cpp (validation, binned-SAH build, the five node layouts, packing, the
host FP32 traversal) is compiled for the host alone with both sanitizers and
driven by tests/host_sanitize/driver.cpp: random scenes of every kind (spheres
only, triangles only with a zero-area and duplicate triangles, mixed with
planes, a single primitive, planes only), leaf sizes 1, 4 and 15, every node
layout, closest-hit and any-hit host traversal (every layout must answer every
query alike), and the validation and depth-limit errors.  Any sanitizer
report aborts the driver.  No GPU call is made; the device half of refit.cpp
(which scene.cpp calls for the refit order) is linked unsanitized.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1504_03151_amd", "csrc")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
HIPCC = os.path.join(ROCM, "bin", "hipcc")
CLANGXX = os.path.join(ROCM, "lib", "llvm", "bin", "clang++")
INC = [f"-I{os.path.join(ROOT, 'include')}", f"-I{CSRC}"]
HOST_SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=all"]


@pytest.mark.slow
def test_host_code_is_clean_under_asan_and_ubsan(tmp_path):
    if not (os.path.exists(HIPCC) and os.path.exists(CLANGXX)):
        pytest.skip("ROCm compilers not found")
    out = str(tmp_path)
    common = ["-O1", "-g", "-std=c++17", "-fno-omit-frame-pointer"] + INC
    steps = [
        [HIPCC, "-x", "hip", "--cuda-host-only"] + common + HOST_SAN +
        ["-c", os.path.join(CSRC, "scene.cpp"), "-o", os.path.join(out, "scene.o")],
        [HIPCC, "-x", "c++"] + common + HOST_SAN +
        ["-c", os.path.join(ROOT, "tests", "host_sanitize", "driver.cpp"), "-o", os.path.join(out, "driver.o")],
        [HIPCC, "-x", "hip", "-O1", "-std=c++17", "-fPIC", "--offload-arch=gfx950", "-Xclang", "-target-feature",
         "-Xclang", "-packed-fp32-ops"] + INC + ["-c", os.path.join(CSRC, "refit.cpp"), "-o", os.path.join(out, "refit.o")],
        [CLANGXX, "-fsanitize=address,undefined", os.path.join(out, "driver.o"), os.path.join(out, "scene.o"),
         os.path.join(out, "refit.o"), "-o", os.path.join(out, "driver"), f"-L{os.path.join(ROCM, 'lib')}",
         "-lamdhip64", f"-Wl,-rpath,{os.path.join(ROCM, 'lib')}"],
    ]
    for cmd in steps:
        r = subprocess.run(cmd, capture_output=True, text=True)
        assert r.returncode == 0, f"{' '.join(cmd)}\n{r.stderr[-3000:]}"
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:halt_on_error=1:abort_on_error=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", HIP_VISIBLE_DEVICES="")
    r = subprocess.run([os.path.join(out, "driver")], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-6000:]
    assert "0 failures" in r.stdout
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr[-3000:]
