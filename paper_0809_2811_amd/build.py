"""Build libsw.so (HIP, gfx950) in-tree with hipcc."""
from __future__ import annotations

import os
import pathlib
import shutil
import subprocess

PKG = pathlib.Path(__file__).resolve().parent
ROOT = PKG.parent
CSRC = PKG / "csrc"
LIB = PKG / "libsw.so"
SOURCES = ["sw_kernels.hip", "sw_tangent.hip", "sw_api.hip", "sw_observe.hip", "sw_npt.hip", "sw_noalloc.hip"]

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-ffp-contract=on",  # fuse only within an expression: every kernel variant rounds alike
    # never emit packed FP32 (v_pk_*_f32) instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and pathlib.Path(cand).exists():
            return cand
    raise RuntimeError("hipcc not found")


def build(verbose: bool = False, extra=()) -> pathlib.Path:
    cmd = [hipcc(), *HIPCC_FLAGS, *extra, f"-I{ROOT / 'include'}", f"-I{CSRC}", "-o", str(LIB)]
    cmd += [str(CSRC / s) for s in SOURCES]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
