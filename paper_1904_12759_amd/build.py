"""Build libmcexpmv.so (HIP, gfx950) in-tree with hipcc.

Usage: python -m paper_1904_12759_amd.build   (or call build()).
Every call recompiles all sources (this is the "does it build" check).
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libmcexpmv.so")
BUILD_DIR = os.path.join(HERE, "_build")

SOURCES = ["api.hip", "setup.hip", "walk.hip", "batch.hip", "mlp.hip", "forward.hip", "isim.hip",
           "sort.hip"]

HIPCC_FLAGS = [
    "-x", "hip", "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # keep the arithmetic op-for-op as written (no fused multiply-add contraction)
    "-ffp-contract=off",
    # no packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"),
    "-Wall", "-Wno-unused-function",
]


def _hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if c and (os.path.isabs(c) and os.path.exists(c) or not os.path.isabs(c)):
            return c
    return "hipcc"


# Host-code sanitizer build (libmcexpmv_san.so, CPU checks only): AddressSanitizer
# and UndefinedBehaviorSanitizer on the host side of every source; device code is
# built as usual.
SAN_LIB = os.path.join(HERE, "libmcexpmv_san.so")
SAN_BUILD_DIR = os.path.join(HERE, "_build_san")
SAN_FLAGS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=all"]


def _compile(src: str, san: bool = False) -> str:
    bdir = SAN_BUILD_DIR if san else BUILD_DIR
    obj = os.path.join(bdir, os.path.splitext(src)[0] + ".o")
    cmd = [_hipcc(), *HIPCC_FLAGS, *(SAN_FLAGS if san else []), "-c", os.path.join(CSRC, src),
           "-o", obj]
    subprocess.run(cmd, check=True, cwd=bdir)
    return obj


def build(verbose: bool = False, sanitize: bool = False) -> str:
    bdir, lib = (SAN_BUILD_DIR, SAN_LIB) if sanitize else (BUILD_DIR, LIB)
    os.makedirs(bdir, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        objs = list(ex.map(lambda src: _compile(src, sanitize), SOURCES))
    tmp = lib + ".tmp"
    cmd = [_hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp]
    subprocess.run(cmd, check=True, cwd=bdir)
    os.replace(tmp, lib)
    if verbose:
        print("built", lib)
    return lib


if __name__ == "__main__":
    build(verbose=True, sanitize="--sanitize" in sys.argv[1:])
    sys.exit(0)
