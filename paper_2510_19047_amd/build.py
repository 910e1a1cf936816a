"""Compile libtfsc.so (HIP, gfx950) in-tree with hipcc.

    python -m paper_2510_19047_amd.build [--force]
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libtfsc.so")
SOURCES = ["tfsc_api.hip", "tfsc_stat.hip", "tfsc_transform.hip", "tfsc_vjp.hip", "tfsc_follow.hip", "tfsc_tiles.hip"]
HEADERS = ["tfsc_device.hpp", "tfsc_kernels.hpp", os.path.join("..", "..", "include", "tfsc.h")]
ARCH = os.environ.get("TFSC_OFFLOAD_ARCH", "gfx950")

FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
    # the FP64 track must be evaluated without contraction (bit-exact bin indices)
    "-ffp-contract=off",
    # never emit packed FP32 arithmetic
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def build(force: bool = True, verbose: bool = False) -> str:
    srcs = [os.path.join(CSRC, s) for s in SOURCES]
    deps = srcs + [os.path.join(CSRC, h) for h in HEADERS]
    if not force and os.path.exists(LIB) and all(os.path.getmtime(LIB) >= os.path.getmtime(d) for d in deps):
        return LIB
    tmp = LIB + ".tmp"
    cmd = ["hipcc", *FLAGS, "-o", tmp, *srcs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd, cwd=CSRC)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(force="--force" in sys.argv or True, verbose=True)
    print(LIB)
