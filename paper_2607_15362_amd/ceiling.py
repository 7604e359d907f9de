"""Binding of the bandwidth instruments (include/goc_ceiling.h, libgocceiling.so):
argument marshalling only.

    python -m paper_2607_15362_amd.ceiling [NX NY MHD STORAGE_BYTES ROWS NT [COLS]]

prints the same-pattern time of the tiled step (default: the 4096 x 1024
Hartmann layout, FP32, D2Q5 slots, 64 x 4 tiles, non-temporal stores) and a
1 GiB one-stream copy as one JSON line;

    python -m paper_2607_15362_amd.ceiling mix

prints one JSON line per read / write mix of plain 1 GiB streams (reads
only, writes only, 1:1, 2:1, 1:2, 2:2), swept grid-stride or in one
contiguous share per work-group, plain and non-temporal stores, at 2 to 32
work-groups per compute unit.
"""
from __future__ import annotations

import ctypes as C
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgocceiling.so")

SIGNATURES = {
    "goc_ceiling_pattern": (C.c_int, [C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int,
                                      C.c_void_p, C.POINTER(C.c_double)]),
    "goc_ceiling_copy": (C.c_int, [C.c_int64, C.c_int, C.c_void_p, C.POINTER(C.c_double)]),
    "goc_ceiling_mix": (C.c_int, [C.c_int64, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.c_void_p,
                                  C.POINTER(C.c_double)]),
}

_lib = None


def lib():
    """Load libgocceiling.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_2607_15362_amd.build.build()")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(rc: int, what: str):
    if rc != 0:
        raise RuntimeError(f"{what} failed with status {rc}")


def pattern_us(nx: int, ny: int, mhd: bool, storage_bytes: int, rows: int, nontemporal: bool, reps: int = 200,
               stream: int = 0, cols: int = 64) -> float:
    """Mean microseconds per launch of the tiled step's memory pattern."""
    out = C.c_double(0.0)
    _check(lib().goc_ceiling_pattern(nx, ny, int(bool(mhd)), storage_bytes, cols, rows, int(bool(nontemporal)),
                                     reps, C.c_void_p(stream or None), C.byref(out)), "goc_ceiling_pattern")
    return out.value


def copy_us(nbytes: int, reps: int = 50, stream: int = 0) -> float:
    """Mean microseconds per launch of a one-stream copy of nbytes."""
    out = C.c_double(0.0)
    _check(lib().goc_ceiling_copy(nbytes, reps, C.c_void_p(stream or None), C.byref(out)), "goc_ceiling_copy")
    return out.value


def mix_us(nbytes: int, reads: int, writes: int, nontemporal: bool = False, wg_per_cu: int = 32, reps: int = 20,
           stream: int = 0, chunked: bool = False) -> float:
    """Mean microseconds per launch of plain streams: `reads` inputs and
    `writes` outputs of nbytes each, swept grid-stride or (chunked) in one
    contiguous share per work-group."""
    out = C.c_double(0.0)
    _check(lib().goc_ceiling_mix(nbytes, reads, writes, int(bool(nontemporal)), int(bool(chunked)), wg_per_cu, reps,
                                 C.c_void_p(stream or None), C.byref(out)), "goc_ceiling_mix")
    return out.value


def mix_table(nbytes: int = 1 << 30):
    """One record per read / write mix, sweep order, store policy and launch
    width."""
    rows = []
    for reads, writes in ((1, 0), (2, 0), (0, 1), (0, 2), (1, 1), (2, 1), (1, 2), (2, 2)):
        for chunked in (False, True):
            for nt in ((False,) if writes == 0 else (False, True)):
                for wg in (2, 4, 8, 16, 32):
                    us = mix_us(nbytes, reads, writes, nt, wg, chunked=chunked)
                    moved = (reads + writes) * nbytes
                    rows.append({"reads": reads, "writes": writes, "chunked": int(chunked), "nontemporal": int(nt),
                                 "wg_per_cu": wg, "us_per_launch": round(us, 2),
                                 "GB_s": round(moved / (us * 1e-6) / 1e9, 1)})
    return rows


def main(argv):
    if argv[:1] == ["mix"]:
        for row in mix_table():
            print(json.dumps(row), flush=True)
        return
    vals = [int(v) for v in argv] if argv else [4096, 1024, 1, 4, 4, 1]
    nx, ny, mhd, sb, rows, nt = vals[:6]
    cols = vals[6] if len(vals) > 6 else 64
    us = pattern_us(nx, ny, bool(mhd), sb, rows, bool(nt), cols=cols)
    nb = 1 << 30
    cu = copy_us(nb)
    print(json.dumps({"pattern": {"nx": nx, "ny": ny, "mhd": mhd, "storage_bytes": sb, "cols": cols, "rows": rows,
                                  "nontemporal": nt, "us_per_launch": round(us, 2)},
                      "copy": {"bytes": nb, "us_per_launch": round(cu, 2),
                               "GB_s_read_plus_write": round(2 * nb / (cu * 1e-6) / 1e9, 1)}}), flush=True)


if __name__ == "__main__":
    main(sys.argv[1:])
