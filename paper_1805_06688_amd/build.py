"""Build libmgrit.so (HIP kernels for gfx950 + host driver + host set-up) in-tree.

    python -m paper_1805_06688_amd.build
"""
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
OUT_DIR = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libmgrit.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
# Packed-FP32 instructions are disabled for every device compilation.
DEVICE_FLAGS = ["-O3", "-fPIC", "-std=c++17", f"--offload-arch={ARCH}",
                "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                "-I", os.path.join(ROOT, "include"), "-I", CSRC]


def _run(cmd):
    print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)


def build(verbose=True):
    os.makedirs(OUT_DIR, exist_ok=True)
    objs = []
    # host-only set-up in binary128 (libquadmath): host compiler
    o = os.path.join(OUT_DIR, "toeplitz_setup.o")
    _run(["g++", "-O2", "-fPIC", "-std=gnu++17", "-I", CSRC, "-c", os.path.join(CSRC, "toeplitz_setup.cpp"), "-o", o])
    objs.append(o)
    o = os.path.join(OUT_DIR, "fd_setup.o")
    _run(["g++", "-O3", "-fPIC", "-std=gnu++17", "-I", CSRC, "-c", os.path.join(CSRC, "fd_setup.cpp"), "-o", o])
    objs.append(o)
    o = os.path.join(OUT_DIR, "kernels.o")
    _run([HIPCC] + DEVICE_FLAGS + ["-c", os.path.join(CSRC, "kernels.hip"), "-o", o])
    objs.append(o)
    for src in ("mgrit_driver.cpp", "server.cpp"):
        o = os.path.join(OUT_DIR, src.replace(".cpp", ".o"))
        _run([HIPCC] + DEVICE_FLAGS + ["-x", "hip", "-c", os.path.join(CSRC, src), "-o", o])
        objs.append(o)
    tmp = LIB + ".tmp"
    _run([HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp] + objs + ["-lquadmath", "-lpthread"])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build()
    sys.exit(0)
