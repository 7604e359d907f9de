"""Build libgoclbm.so for gfx950 with hipcc (in-tree, no JIT cache)."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libgoclbm.so")
SOURCES = [os.path.join(CSRC, "goc_lbm.hip")]
DEPS = SOURCES + [os.path.join(CSRC, f) for f in ("goc_device.hpp", "goc_step.hpp", "goc_tile.hpp", "goc_aux.hpp")] + [
    os.path.join(os.path.dirname(HERE), "include", "goc_lbm.h")]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"


def flags():
    return ["--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC", "-shared",
            "-munsafe-fp-atomics",
            # packed FP32 instructions are disabled for all device code
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wno-unused-command-line-argument"]


def build(force: bool = True, verbose: bool = False) -> str:
    """Compile the library; force=True always recompiles."""
    if not force and os.path.exists(LIB):
        t = os.path.getmtime(LIB)
        if all(os.path.getmtime(d) <= t for d in DEPS):
            return LIB
    tmp = LIB + ".tmp"
    cmd = [HIPCC] + flags() + ["-o", tmp] + SOURCES
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(force=True, verbose=True)
    sys.exit(0)
