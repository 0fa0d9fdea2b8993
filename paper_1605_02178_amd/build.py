"""Build libbfgc.so (HIP for gfx950) in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libbfgc.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
# Packed FP32 instructions are kept out of the generated code.
DEVICE_FLAGS = ["--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def build(verbose: bool = False, extra: list[str] | None = None) -> str:
    tmp = LIB + ".tmp"
    obj = os.path.join(CSRC, "plan.o")
    # The host planner uses binary128 (libquadmath), which g++ provides.
    cc = ["g++", "-O2", "-std=gnu++17", "-fPIC", "-Wall", "-c", os.path.join(CSRC, "plan.cpp"), "-o", obj]
    dobj = os.path.join(CSRC, "bfgc.o")
    dev = [HIPCC, "-O3", "-std=c++17", "-fPIC", *DEVICE_FLAGS,
           "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-Wall", "-Wno-unused-function",
           *(extra or []), "-c", os.path.join(CSRC, "bfgc.hip"), "-o", dobj]
    link = [HIPCC, "-shared", "-fPIC", "--hip-link", "--offload-arch=gfx950", dobj, obj, "-lquadmath", "-o", tmp]
    for c in (cc, dev, link):
        if verbose:
            print(" ".join(c), flush=True)
        subprocess.run(c, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
