"""Hardware-rate microbenchmarks on the current GPU (gfx950): LDS FP32/FP64
and 32/64-bit integer atomic adds and reads under several lane-to-address
patterns, global FP64
atomic adds, and HBM copy bandwidth.  ``python -m
paper_2303_12873_amd.microbench`` prints one JSON line per measurement.

The kernels are in ``csrc/pic_microbench.hip`` (library ``libpic_mb.so``).
"""
from __future__ import annotations

import ctypes as C
import json
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
MB_PATH = os.path.join(_HERE, "libpic_mb.so")
PATTERNS = {0: "distinct consecutive", 1: "4 lanes per slot", 2: "whole wave one slot",
            3: "distinct, 2-word stride", 4: "distinct, 15-word stride",
            5: "8x8 cells, row 15", 6: "8x8 cells, row 24", 7: "16x4 cells, row 23",
            8: "16x4 cells, row 24", 9: "16x4 cells, row 23, lane bits 4/5 swapped",
            10: "16x4 cells, row 24, lane bits 4/5 swapped"}


def _lib():
    if not os.path.exists(MB_PATH):
        raise RuntimeError(f"{MB_PATH} is not built: run `python -m paper_2303_12873_amd.build`")
    L = C.CDLL(MB_PATH)
    L.pic_mb_lds.argtypes = [C.c_int] * 5
    L.pic_mb_lds.restype = C.c_float
    L.pic_mb_global_atomic.argtypes = [C.c_longlong, C.c_longlong, C.c_int, C.c_int]
    L.pic_mb_global_atomic.restype = C.c_float
    L.pic_mb_copy.argtypes = [C.c_longlong, C.c_int]
    L.pic_mb_copy.restype = C.c_float
    return L


def run(cus: int = 256):
    L = _lib()
    out = []
    blocks, iters = cus * 4, 256
    for kind, kname in ((0, "lds_atomic_add"), (1, "lds_read"), (2, "lds_atomic_add_int")):
        for nbytes in (4, 8):
            for pat in PATTERNS:
                ms = L.pic_mb_lds(kind, nbytes, pat, blocks, iters)
                wave_ops = blocks * (512 // 64) * iters * 8
                out.append({"test": kname, "bytes": nbytes, "pattern": PATTERNS[pat], "ms": ms,
                            "wave_ops_per_s": wave_ops / (ms * 1e-3),
                            "cycles_per_wave_op_per_cu": (ms * 1e-3 * 2.4e9 * cus) / wave_ops})
    for collide in (0, 1):
        threads, iters = 1 << 22, 64
        ms = L.pic_mb_global_atomic(threads, 1 << 24, iters, collide)
        out.append({"test": "global_atomic_add_f64", "pattern": "one slot per wave" if collide else "distinct",
                    "ms": ms, "atomics_per_s": threads * iters / (ms * 1e-3)})
    nbytes = 4 << 30
    ms = L.pic_mb_copy(nbytes, cus * 16)
    out.append({"test": "hbm_copy", "bytes": nbytes, "ms": ms, "GB_per_s": 2 * nbytes / (ms * 1e-3) / 1e9})
    return out


def copy_only(nbytes: int = 4 << 30, cus: int = 256):
    """One timed device copy of nbytes (the calibration run for HBM counters)."""
    ms = _lib().pic_mb_copy(nbytes, cus * 16)
    return {"test": "hbm_copy", "bytes": nbytes, "ms": ms, "GB_per_s": 2 * nbytes / (ms * 1e-3) / 1e9}


if __name__ == "__main__":
    import sys
    rows = [copy_only()] if sys.argv[1:] == ["copy"] else run()
    for r in rows:
        print(json.dumps(r), flush=True)
