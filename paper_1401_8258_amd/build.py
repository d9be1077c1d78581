"""Compile libdedisp.so for gfx950 in-tree (hipcc cross-compiles without a GPU)."""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
SRC = [os.path.join(PKG, "csrc", "dedisp.hip"), os.path.join(PKG, "csrc", "regwin.hip"),
       os.path.join(PKG, "csrc", "direct.hip"),
       os.path.join(PKG, "csrc", "detrend.hip"),
       os.path.join(PKG, "csrc", "boxcar.hip"), os.path.join(PKG, "csrc", "downfactor.hip"),
       os.path.join(PKG, "csrc", "rfi.hip"),
       os.path.join(PKG, "csrc", "plan.cpp")]
LIB = os.path.join(PKG, "libdedisp.so")

FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "-shared", "--offload-arch=gfx950",
    # one rounding per double operation in the host delay table, no FMA contraction anywhere
    "-ffp-contract=off",
    # packed FP32 VALU forms are kept out of the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if cand and (os.path.isabs(cand) and os.path.exists(cand) or not os.path.isabs(cand)):
            return cand
    return "hipcc"


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp"
    cmd = [hipcc()] + FLAGS + SRC + ["-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed building libdedisp.so")
    if verbose:
        sys.stderr.write(r.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
