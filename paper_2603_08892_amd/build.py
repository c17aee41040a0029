"""Build libns.so (HIP, gfx950) in-tree.

    python -m paper_2603_08892_amd.build          # or build() from Python

hipcc cross-compiles without a GPU.  Packed FP32 instructions are disabled
(-packed-fp32-ops) for every HIP translation unit.
"""

import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libns.so")
SOURCES = [os.path.join(CSRC, "ns_host.hip")]
HEADERS = [os.path.join(CSRC, f) for f in ("fft_core.hpp", "ns_kernels.hpp", "ns_aux_kernels.hpp", "ns_adjoint.hpp", "fft_reg.hpp", "ns_fast.hpp", "ns_fast_adjoint.hpp", "ns_model1d.hpp")] + [
    os.path.join(ROOT, "include", "ns.h")]


def hipcc():
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found (ROCm is required to build libns.so)")


def command(out=LIB, extra=()):
    return [hipcc(), "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wno-unused-command-line-argument",
            "-I", os.path.join(ROOT, "include"), *extra, "-o", out, *SOURCES]


def build(verbose=True):
    """Compile libns.so every time it is called (atomic replace of the old file)."""
    tmp = LIB + ".tmp"
    cmd = command(tmp)
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
