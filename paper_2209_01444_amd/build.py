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
SUR_DEPS = SUR_SOURCES + [os.path.join(ROOT, "include", "sur.h")]

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


def stale(lib: str = LIB, deps=None) -> bool:
    """True if the library is missing or older than any of its sources."""
    if not os.path.exists(lib):
        return True
    t = os.path.getmtime(lib)
    return any(os.path.getmtime(d) > t for d in (DEPS if deps is None else deps))


def warn_if_stale(lib: str, deps) -> None:
    """Say so on stderr when a library is older than its sources: it still
    loads (a copied tree may not keep modification times), but it may not be
    the code the sources describe."""
    if os.path.exists(lib) and stale(lib, deps):
        newer = [os.path.basename(d) for d in deps if os.path.getmtime(d) > os.path.getmtime(lib)]
        print(f"warning: {lib} is older than {', '.join(newer)}; rebuild with "
              "`python paper_2209_01444_amd/build.py`", file=sys.stderr, flush=True)


if __name__ == "__main__":
    print(build(verbose=True))
    sys.exit(0)
