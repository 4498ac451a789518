"""The C ABI's host code under AddressSanitizer and UndefinedBehaviorSanitizer
(CPU only).  The library's sources are compiled with host-side
instrumentation (device code is built as usual and not run) and linked with
tests/abi_check.c, which drives every host-side validation and argument
check of include/halp.h: malformed LPs and options, NULL handles, a
randomised sweep of malformed CSR input and the canonicalisation of
unsorted / duplicate column indices.  Any out-of-bounds access,
use-after-free or undefined behaviour aborts the program (leak checks
are off: the HIP runtime keeps allocations until exit)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2407_16144_amd", "csrc")
HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"

ARCH = f"--offload-arch={os.environ.get('HALP_OFFLOAD_ARCH', 'gfx950')}"
INCLUDES = [f"-I{os.path.join(ROOT, 'include')}", f"-I{CSRC}"]
# the library's own device flags (packed FP32 off), as in its normal build
HIP_FLAGS = ["-std=c++17", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-Wno-unused-result"]
# host-side instrumentation only: each sanitizer flag applies to the host pass
HOST_SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer"]


@pytest.mark.timeout(600)
def test_abi_host_code_under_sanitizers(tmp_path):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    units = [(os.path.join(CSRC, "engine.hip"), HIP_FLAGS), (os.path.join(CSRC, "abi.cpp"), HIP_FLAGS),
             (os.path.join(ROOT, "tests", "abi_check.c"), ["-x", "c", "-std=c99"])]
    objs = []
    for src, flags in units:
        obj = str(tmp_path / (os.path.basename(src) + ".o"))
        subprocess.run([HIPCC, "-O1", "-g", ARCH] + flags + INCLUDES + HOST_SAN + ["-c", src, "-o", obj],
                       check=True, capture_output=True)
        objs.append(obj)
    exe = str(tmp_path / "abi_check")
    subprocess.run([HIPCC, ARCH, "-fsanitize=address,undefined", "-fno-gpu-sanitize"] + objs + ["-o", exe],
                   check=True, capture_output=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    p = subprocess.run([exe], env=env, capture_output=True, text=True, timeout=300)
    assert p.returncode == 0, p.stdout[-2000:] + p.stderr[-4000:]
    assert "abi checks passed" in p.stdout
