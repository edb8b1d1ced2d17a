"""Build libmpdet.so (hand-written HIP for gfx950) in-tree with hipcc.

    python -m paper_1308_1536_amd.build          # builds paper_1308_1536_amd/libmpdet.so

The library is compiled for gfx950 only, with packed-FP32 instruction
selection disabled (the kernels use integer arithmetic; the flag keeps the
compiler from emitting packed FP32 forms anywhere).
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libmpdet.so")
SOURCES = [os.path.join(CSRC, "mpdet_api.hip")]
ARCH = "gfx950"


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found (ROCm is required to build libmpdet.so)")


def command(out: str = LIB, extra: list[str] | None = None) -> list[str]:
    return [hipcc(), "-O3", "-std=c++17", f"--offload-arch={ARCH}", "-fPIC", "-shared",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wall", "-Wno-unused-function",
            "-I", INCLUDE, "-I", CSRC, *SOURCES, "-o", out, *(extra or [])]


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp"
    cmd = command(tmp)
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
