"""The host code of libmgrit under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only, no GPU).

Builds the host set-up sources (binary128 Toeplitz sequences, the preconditioner's eigen-solver) with g++
and the HIP driver and server with the sanitizers on their host side only (`-Xarch_host` before each
`-fsanitize=`), links them with the kernels into a test program (tests/sanitize/host_checks.cpp) and runs
it: every check must pass and the sanitizers must find nothing (they abort on their first finding).  The
link uses the GNU sanitizer runtimes, so clang's function-type check (no GNU counterpart) is left out.
Leak checking is off: the HIP runtime keeps allocations of its own until exit.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1805_06688_amd", "csrc")
INC = os.path.join(ROOT, "include")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

pytestmark = pytest.mark.slow


def _run(cmd, cwd):
    r = subprocess.run(cmd, cwd=cwd, capture_output=True, text=True)
    assert r.returncode == 0, (cmd, r.stdout[-2000:], r.stderr[-4000:])
    return r


@pytest.mark.skipif(not os.path.exists(HIPCC) or shutil.which("g++") is None, reason="needs hipcc and g++")
def test_host_code_is_clean_under_asan_and_ubsan(tmp_path):
    san = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]
    hsan = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize=function", "-Xarch_host", "-fno-sanitize-recover=all"]
    dev = ["-O1", "-g", "-fPIC", "-std=c++17", "--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang",
           "-packed-fp32-ops", "-I", INC, "-I", CSRC]
    d = str(tmp_path)
    for src in ("toeplitz_setup.cpp", "fd_setup.cpp"):
        _run(["g++", "-O1", "-g", "-std=gnu++17"] + san + ["-I", CSRC, "-c", os.path.join(CSRC, src), "-o",
                                                          src + ".o"], d)
    for src in ("mgrit_driver.cpp", "server.cpp"):
        _run([HIPCC] + dev + hsan + ["-x", "hip", "-c", os.path.join(CSRC, src), "-o", src + ".o"], d)
    _run([HIPCC] + dev + ["-c", os.path.join(CSRC, "kernels.hip"), "-o", "kernels.o"], d)
    _run(["g++", "-O1", "-g"] + san + ["-I", INC, "-c", os.path.join(ROOT, "tests", "sanitize", "host_checks.cpp"),
                                       "-o", "main.o"], d)
    _run(["g++"] + san + ["main.o", "mgrit_driver.cpp.o", "server.cpp.o", "toeplitz_setup.cpp.o", "fd_setup.cpp.o",
                          "kernels.o", "-L/opt/rocm/lib", "-Wl,-rpath,/opt/rocm/lib", "-lamdhip64", "-lquadmath",
                          "-lpthread", "-o", "host_checks"], d)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1",
               HIP_VISIBLE_DEVICES="")
    r = subprocess.run([os.path.join(d, "host_checks")], cwd=d, env=env, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, (r.stdout[-3000:], r.stderr[-6000:])
    assert "0 failures" in r.stdout
