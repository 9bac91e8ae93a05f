"""Build libdlb.so for gfx950 in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIBDIR = os.path.join(HERE, "_lib")
LIB = os.path.join(LIBDIR, "libdlb.so")
SOURCES = [os.path.join(CSRC, "dlb.hip"), os.path.join(CSRC, "dlb3.hip")]
DEPS = SOURCES + [os.path.join(CSRC, f) for f in ("lattice.h", "kernels.h", "batch.h")] + [
    os.path.join(ROOT, "include", "dlb.h"), os.path.join(ROOT, "include", "dlb3.h")]
SUR_LIB = os.path.join(LIBDIR, "libsur.so")
SUR_SOURCES = [os.path.join(CSRC, "sur.hip")]

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # packed FP32 instructions are kept out of every kernel
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def hipcc() -> str:
    return os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def _compile(sources, lib, verbose):
    tmp = lib + ".tmp"
    cmd = [hipcc(), *HIPCC_FLAGS, "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-o", tmp, *sources]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, lib)
    return lib


def build(verbose: bool = False) -> str:
    """Compile libdlb.so (lattice Boltzmann solver) and libsur.so (surrogate)."""
    os.makedirs(LIBDIR, exist_ok=True)
    _compile(SUR_SOURCES, SUR_LIB, verbose)
    return _compile(SOURCES, LIB, verbose)


def stale() -> bool:
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    return any(os.path.getmtime(d) > t for d in DEPS)


if __name__ == "__main__":
    print(build(verbose=True))
    sys.exit(0)
