"""Compile the HIP library libqedspin.so for gfx950 (in-tree, next to this file)."""
from __future__ import annotations

import os
import subprocess
import sys
from pathlib import Path

PKG = Path(__file__).resolve().parent
CSRC = PKG / "csrc"
INCLUDE = PKG.parent / "include"
LIB = PKG / "libqedspin.so"
SOURCES = ["qs_tables.hip", "qs_step.hip", "qs_plan.hip", "qs_mlp.hip", "qs_profile.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC", "-shared",
         # FP32 division and square root by the hardware approximations (FP64 is unaffected)
         "-fno-hip-fp32-correctly-rounded-divide-sqrt",
         # FP32 denormals flushed to zero (FP64 keeps them): the single-precision values of the
         # step are far from 1e-38, and reciprocals, square roots and exponentials then need no
         # rescaling around the hardware instructions
         "-fgpu-flush-denormals-to-zero",
         # fused multiply-add only where one source expression has the form a*b+c: the same
         # function inlined into different kernels then rounds the same way, so the per-species
         # calls and the merged step agree bit for bit
         "-ffp-contract=on",
         # keep packed FP32 instructions out of the generated code
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-function", "-Wno-unused-variable"]


def build(verbose: bool = False) -> Path:
    tmp = LIB.with_suffix(".so.tmp")
    cmd = [HIPCC, *FLAGS, f"-I{INCLUDE}", "-o", str(tmp)] + [str(CSRC / s) for s in SOURCES]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(LIB)
