"""Hardware-rate microbenchmarks on the current GPU (gfx950): LDS FP32/FP64
and 32/64-bit integer atomic adds and reads under several lane-to-address
patterns, global FP64
atomic adds, HBM copy bandwidth and the field-stage copy.  ``python -m
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
    L.pic_mb_stage_rows.argtypes = [C.c_int] * 6
    L.pic_mb_stage_rows.restype = C.c_double
    L.pic_mb_stage_rows_w.argtypes = [C.c_int] * 8 + [C.POINTER(C.c_float)]
    L.pic_mb_stage_rows_w.restype = C.c_double
    return L


def stage_width(cus: int = 256, rows: int = 390, length: int = 24, row_stride: int = 256,
                reps: int = 8, lds_off: int = 0):
    """The field-stage copy with 4, 12 or 16 bytes per lane (one, three or
    four dwords of a row per lane), rows of `length` floats starting 116
    bytes into a 128-byte line (112 for 16 bytes, which need 16-byte
    alignment), landing at LDS word `lds_off` on.  Checks that workgroup
    0's LDS words equal the source (row r, element j at r * row_stride +
    start + j) and reports the time."""
    L = _lib()
    out = []
    for width, start in ((4, 29), (12, 29), (16, 28)):
        chk = (C.c_float * (rows * length))()
        ticks = L.pic_mb_stage_rows_w(width, cus, rows, length, start, row_stride, reps, lds_off,
                                      chk)
        bad = sum(1 for r in range(rows) for j in range(length)
                  if chk[r * length + j] != float(r * row_stride + start + j))
        out.append({"test": "stage_width", "bytes_per_lane": width, "blocks": cus, "rows": rows,
                    "floats_per_row": length, "start_byte_in_line": start * 4 % 128, "reps": reps,
                    "us_per_stage": ticks / 100.0, "bytes": rows * length * 4,
                    "lds_byte_offset": lds_off * 4, "layout_mismatches": bad})
    return out


def stage_rows(cus: int = 256, rows: int = 390, row_stride: int = 256, reps: int = 8):
    """The field-stage copy: one 1024-thread workgroup per CU copies `rows`
    row segments (1 KB apart, as the x rows of a 256-wide box) into LDS with
    global -> LDS loads, `reps` times.  Segments of 21 floats (the order-3
    16-wide tile's rows) starting 12 bytes before a 128-byte line touch two
    lines, starting on a line one; 32 floats on a line fill it; 16 floats
    fill half of one.  Time per stage against lines per stage tells whether
    the copy is bound by line requests or by bytes or instructions."""
    L = _lib()
    out = []
    for length, start in ((21, 29), (21, 0), (32, 0), (16, 0), (42, 29)):
        first = start * 4 // 128
        last = (start + length) * 4 - 1
        lines_per_row = last // 128 - first + 1
        ticks = L.pic_mb_stage_rows(cus, rows, length, start, row_stride, reps)
        us = ticks / 100.0
        out.append({"test": "stage_rows", "rows": rows, "floats_per_row": length,
                    "start_byte_in_line": start * 4 % 128, "lines_per_row": lines_per_row,
                    "lines": rows * lines_per_row, "bytes": rows * length * 4, "reps": reps,
                    "us_per_stage": us,
                    "ns_per_line": us * 1e3 / (rows * lines_per_row) if ticks > 0 else None})
    return out


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
    if sys.argv[1:] == ["copy"]:
        rows = [copy_only()]
    elif sys.argv[1:] == ["stage"]:
        # the last: copies landing from 64 KB of LDS on
        rows = (stage_rows() + stage_width(cus=8) + stage_width() +
                stage_width(cus=8, rows=200, lds_off=16384))
    else:
        rows = (run() + stage_rows() + stage_width(cus=8) + stage_width() +
                stage_width(cus=8, rows=200, lds_off=16384))
    for r in rows:
        print(json.dumps(r), flush=True)
