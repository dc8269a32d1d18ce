"""Build the HIP library libd2q37.so in-tree with hipcc for gfx950.

Usage: python -m paper_1703_00185_amd.build   (or build() from Python).
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libd2q37.so")
SOURCES = [os.path.join(CSRC, "kernels.hip"), os.path.join(CSRC, "engine.hip"),
           os.path.join(CSRC, "lbm_api.cpp"), os.path.join(CSRC, "engine_api.cpp"),
           os.path.join(CSRC, "noalloc_api.cpp")]
ARCH = "gfx950"

# -ffp-contract=off: every fused multiply-add in the kernels is an explicit
# fma(); the host-side wall factors must round as written.
# -packed-fp32-ops: packed FP32 instructions are disabled on this target.
FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "-shared", f"--offload-arch={ARCH}",
    "-ffp-contract=off", "-Wall", "-Wno-unused-function",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def build(verbose: bool = False, extra_flags: list[str] | None = None, out: str = LIB) -> str:
    """Compile every HIP/C++ source of the library into `out`; returns its path."""
    tmp = out + ".tmp"
    cmd = [hipcc(), *FLAGS, *(extra_flags or []), "-x", "hip", *SOURCES, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"hipcc failed ({res.returncode}):\n{res.stdout}\n{res.stderr}")
    if verbose and res.stderr.strip():
        print(res.stderr, file=sys.stderr)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
