"""Builds libgicp.so for gfx950 with hipcc (in-tree, next to this file).

    python -m paper_2403_12550_amd.build        # or: python paper_2403_12550_amd/build.py
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libgicp.so")
SOURCES = ["grid.hip", "knn.hip", "gn.hip", "mlp.hip", "depth.hip", "api.hip"]
ARCH = os.environ.get("GICP_OFFLOAD_ARCH", "gfx950")

FLAGS = [
    f"--offload-arch={ARCH}",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    # packed FP32 instructions stay off in the device code (without this flag
    # hipcc -O3 forms v_pk_fma_f32 / v_pk_add_f32 from plain float code for
    # gfx950; with it, none: checked on the assembly of a float2 kernel).  The
    # host pass, which has no such feature, warns that it ignores the flag.
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # fuse multiply-adds only within one expression, so that the same source
    # expression rounds the same way in every kernel that inlines it
    "-ffp-contract=on",
    "-Wall",
    "-Wno-unused-function",
]


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def build(verbose: bool = False) -> str:
    srcs = [os.path.join(CSRC, s) for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    tmp = LIB + ".tmp"
    cmd = [hipcc(), *FLAGS, *srcs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError(f"hipcc failed ({r.returncode})")
    if verbose and r.stderr.strip():
        sys.stderr.write(r.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
