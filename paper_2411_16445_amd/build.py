"""Build of the HIP library libplasticarbor.so (gfx950) in-tree.

    python -m paper_2411_16445_amd.build
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libplasticarbor.so")
SOURCES = ["api.cpp", "kernels.hip", "kernels_fused.hip", "tree_solve.hip", "gb_trials.hip"]
ARCH = os.environ.get("PA_OFFLOAD_ARCH", "gfx950")

# -ffp-contract=off: no FMA contraction, so FP64 arithmetic is that of the
# source read literally (bitwise reproducible against a CPU evaluation of
# the same expressions).  Packed FP32 instructions are disabled.
FLAGS = ["-O3", "-std=c++17", "-fPIC", "-shared", f"--offload-arch={ARCH}",
         "-ffp-contract=off", "-fno-fast-math",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-command-line-argument"]


def build(verbose: bool = False) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tmp = LIB + ".tmp"
    cmd = [hipcc, *FLAGS, "-o", tmp, *[os.path.join(CSRC, s) for s in SOURCES]]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed building libplasticarbor.so")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
