"""Compile libtfsc.so (HIP, gfx950) in-tree with hipcc.

    python -m paper_2510_19047_amd.build [--force]

Each source is compiled to its own object in parallel (they share no device
symbols), then the objects are linked into one shared library.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libtfsc.so")
SOURCES = ["tfsc_api.hip", "tfsc_stat.hip", "tfsc_fresnel.hip", "tfsc_harm.hip", "tfsc_transform.hip", "tfsc_vjp.hip",
           "tfsc_follow.hip", "tfsc_tiles.hip", "tfsc_interleave.hip", "tfsc_links.hip"]
HEADERS = ["tfsc_device.hpp", "tfsc_kernels.hpp", "tfsc_stat_common.hpp", os.path.join("..", "..", "include", "tfsc.h")]
ARCH = os.environ.get("TFSC_OFFLOAD_ARCH", "gfx950")

FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    # the FP64 track must be evaluated without contraction (bit-exact bin indices)
    "-ffp-contract=off",
    # never emit packed FP32 arithmetic
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def _jobs() -> int:
    n = int(os.environ.get("MAX_JOBS", "0") or 0)
    return max(1, min(n if n > 0 else (os.cpu_count() or 1), len(SOURCES), 16))


def build(force: bool = True, verbose: bool = False) -> str:
    srcs = [os.path.join(CSRC, s) for s in SOURCES]
    deps = srcs + [os.path.join(CSRC, h) for h in HEADERS]
    if not force and os.path.exists(LIB) and all(os.path.getmtime(LIB) >= os.path.getmtime(d) for d in deps):
        return LIB
    os.makedirs(OBJ, exist_ok=True)
    objs = [os.path.join(OBJ, os.path.splitext(s)[0] + ".o") for s in SOURCES]

    def compile_one(pair):
        src, obj = pair
        cmd = ["hipcc", *FLAGS, "-c", "-o", obj, src]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd, cwd=CSRC)

    with ThreadPoolExecutor(max_workers=_jobs()) as ex:
        list(ex.map(compile_one, zip(srcs, objs)))
    tmp = LIB + ".tmp"
    cmd = ["hipcc", f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd, cwd=CSRC)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(force=True, verbose="-v" in sys.argv)
    print(LIB)
