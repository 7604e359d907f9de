"""Build libgoclbm.so (the solver) and libgocceiling.so (the bandwidth
instruments of the roofline) for gfx950 with hipcc (in-tree, no JIT cache)."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libgoclbm.so")
SOURCES = [os.path.join(CSRC, "goc_lbm.hip")]
INCLUDE = os.path.join(os.path.dirname(HERE), "include")
HEADERS = [os.path.join(CSRC, f) for f in ("goc_device.hpp", "goc_step.hpp", "goc_tile.hpp", "goc_aux.hpp")]
DEPS = SOURCES + HEADERS + [os.path.join(INCLUDE, "goc_lbm.h")]
CEILING_LIB = os.path.join(HERE, "libgocceiling.so")
CEILING_SOURCES = [os.path.join(CSRC, "goc_ceiling.hip")]
CEILING_DEPS = CEILING_SOURCES + HEADERS + [os.path.join(INCLUDE, "goc_ceiling.h"), os.path.join(INCLUDE, "goc_lbm.h")]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"


def flags():
    return ["--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC", "-shared",
            "-munsafe-fp-atomics",
            # packed FP32 instructions are disabled for all device code
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wno-unused-command-line-argument"]


def _compile(lib: str, sources, deps, force: bool, verbose: bool) -> str:
    if not force and os.path.exists(lib):
        t = os.path.getmtime(lib)
        if all(os.path.getmtime(d) <= t for d in deps):
            return lib
    tmp = lib + ".tmp"
    cmd = [HIPCC] + flags() + ["-o", tmp] + list(sources)
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, lib)
    return lib


def build(force: bool = True, verbose: bool = False) -> str:
    """Compile both libraries; force=True always recompiles.  Returns the
    solver library's path."""
    _compile(CEILING_LIB, CEILING_SOURCES, CEILING_DEPS, force, verbose)
    return _compile(LIB, SOURCES, DEPS, force, verbose)


def build_ceiling(force: bool = False, verbose: bool = False) -> str:
    """Compile the instrument library only (when missing or stale)."""
    return _compile(CEILING_LIB, CEILING_SOURCES, CEILING_DEPS, force, verbose)


if __name__ == "__main__":
    build(force=True, verbose=True)
    sys.exit(0)
