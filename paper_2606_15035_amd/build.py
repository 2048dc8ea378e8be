"""Build the HIP library libecpic.so for gfx950 (in-tree).

    python -m paper_2606_15035_amd.build

Compiles every translation unit under csrc/ with hipcc into one shared
library next to this file.  Packed FP32 instructions are disabled for the
device code (-packed-fp32-ops); FP64 atomics compile to the hardware
instructions (-munsafe-fp-atomics).
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libecpic.so")
SOURCES = ["api.hip", "particles.hip", "mesh.hip", "sort.hip", "adjoint.hip", "anderson.hip",
           "measure.hip"]
ARCH = os.environ.get("ECPIC_OFFLOAD_ARCH", "gfx950")


def hipcc_command(out=LIB):
    return (["hipcc", "-O3", "-std=c++17", f"--offload-arch={ARCH}", "-fPIC", "-shared",
             "-munsafe-fp-atomics", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Wall", "-Wno-unused-function",
             "-I", os.path.join(ROOT, "include"), "-I", CSRC]
            + [os.path.join(CSRC, s) for s in SOURCES] + ["-o", out])


def build(verbose=False) -> str:
    cmd = hipcc_command(LIB + ".tmp")
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    print(LIB)
    sys.exit(0)
