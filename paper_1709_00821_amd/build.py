"""Build the HIP library (gfx950) in-tree: paper_1709_00821_amd/libfdtd_plasma.so."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libfdtd_plasma.so")
SOURCES = ["api.hip", "kernels1d.hip", "blocked1d.hip", "adjoint1d.hip", "fft1d.hip", "api3d.hip",
           "kernels3d.hip", "api2d.hip", "kernels2d.hip"]

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-fPIC", "-shared", "-std=c++17",
    # every multiply-add is either an explicit fma or separately rounded, so
    # all execution modes give identical bits
    "-ffp-contract=off",
    # hand-written packed FP32 is avoided; keep the compiler from forming it too
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
]


def sources():
    return [os.path.join(CSRC, s) for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]


def build(verbose: bool = False, extra=None) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    cmd = [hipcc, *HIPCC_FLAGS, *(extra or []), "-o", LIB + ".tmp", *sources()]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True, extra=sys.argv[1:])
