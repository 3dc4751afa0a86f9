"""Build libdr.so in-tree with hipcc for gfx950.

Flags: -ffp-contract=off keeps every fp32 expression the correctly rounded
result of its written operation sequence (no fused multiply-add), which the
bit-exact reproducibility of the estimator relies on; packed fp32 ops are
disabled.
"""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
SOURCES = [os.path.join(CSRC, "dr_kernels.hip"), os.path.join(CSRC, "dr_api.hip"), os.path.join(CSRC, "dr_subdiv.cpp"),
           os.path.join(CSRC, "dr_probe.hip")]
OUT = os.path.join(HERE, "libdr.so")

HIPCC_FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-ffp-contract=off", "-fPIC", "-shared",
               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
               "-I" + os.path.join(ROOT, "include"), "-I" + CSRC]


def build_lib(verbose: bool = False) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tmp = OUT + ".tmp"
    cmd = [hipcc] + HIPCC_FLAGS + ["-o", tmp] + SOURCES
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build_lib(verbose=True))
