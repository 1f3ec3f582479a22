"""Benchmark of the PIC hot path on one MI355X.

One step = the whole hot path over the workload: per-tile sort (every
``--sort-every`` steps, amortised), fused gather + Boris push + Esirkepov
deposit, and the Yee update, issued as one captured HIP graph launch.  The
headline ``value`` is particle-steps/s of the FP32 split-precision batched
form; the plain FP64 form runs on the same inputs beside it.

Default workload: the largest single-GPU case -- 256x256x2048 cells, electrons
and ions (mass ratio 1836) at 4 each per cell behind a 120-cell vacuum with a
100-cell density ramp, order-3 shapes, a0 = 4 Gaussian laser; inputs are
generated on the device from seeded generators (``pic_inputs``).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "particle-steps/s (gather+push+deposit), FP32+batched vs FP64 plain, 1 GPU"

# Algorithmic work per unit (the design doc derives them): bytes a particle must
# move per step (read x,u,w; write x,u), bytes per cell of E/B read and J
# written by the particle kernel, and flops per particle (FMA = 2) by order.
BYTES_PER_PARTICLE = {"fp64": 104, "fp32": 60, "fp32_2d": 52}
BYTES_PER_CELL = {"fp64": 72, "fp32": 48}
FLOPS_PER_PARTICLE = {1: 550, 2: 1150, 3: 2150}
PEAK_HBM_GBS = 8000.0
PEAK_FP32_TFLOPS = 157.3
PEAK_FP64_TFLOPS = 78.6


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def build_workload(name, device):
    import pic_inputs as pi
    if name == "c5":
        return pi.c5(device)
    if name == "c2":
        return pi.c2(device)
    if name == "c4":
        return pi.c4(device)
    if name == "c1":
        return pi.c1(device)
    if name == "c3":
        return pi.c3(device)
    raise SystemExit(f"unknown workload {name}")


def run_form(wl, precision, kernel, steps, warmup, sort_every, tile, block, chunk, wg, stride):
    import torch
    import paper_2303_12873_amd as pic
    import pic_inputs as pi

    boxes = [pi.Box(b.dim, b.n, b.dt, b.order, tuple(tile) if b.dim == 3 else (tile[0], 1, tile[2]),
                    b.dx) for b in wl.boxes]
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        ctx = pic.pic_init(boxes, precision, stream=stream.cuda_stream, kernel=kernel,
                           block=block, chunk=chunk, wg_per_cu=wg, lane_stride=stride)
        f = pic.make_fields(boxes, wl.E, wl.B, precision)
        sp = [pic.make_species(p, precision) for p in wl.species]
    torch.cuda.synchronize()
    np_tot = sum(s.np for s in sp)

    def one(k):
        pic.pic_step(ctx, f, sp, sort=(k % sort_every == 0))

    t0 = time.time()
    for k in range(warmup):
        one(k)
    torch.cuda.synchronize()
    log(f"  warmup {warmup} steps {time.time() - t0:.2f}s")
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record(stream)
    for k in range(steps):
        one(k)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms_step = ev0.elapsed_time(ev1) / steps
    pic.pic_check(ctx)
    # The particle kernel alone (plus its J clear and queue reset): the
    # dominant kernel for the roofline figures.
    nrep = max(3, min(10, steps))
    pic.pic_sort_tiles(ctx, sp)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(nrep):
        pic.pic_advance(ctx, f, sp)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_adv = e0.elapsed_time(e1) / nrep
    # and the sort alone
    e0.record(stream)
    pic.pic_sort_tiles(ctx, sp)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_sort = e0.elapsed_time(e1)
    e0.record(stream)
    pic.pic_fdtd_step(ctx, f)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_fdtd = e0.elapsed_time(e1)
    pic.pic_check(ctx)
    pic.pic_free(ctx)
    del f, sp
    torch.cuda.empty_cache()
    return dict(np=np_tot, ms_step=ms_step, ms_advance=ms_adv, ms_sort=ms_sort, ms_fdtd=ms_fdtd,
                cells=sum(b.ncells for b in boxes))


def cpu_baseline(workload, order):
    """The FP64 oracle, single-threaded, on a bounded sample of the same
    workload: the same transverse structure at a quarter of the transverse
    size, particles restricted to 8 cell layers of the plateau (z 220..228),
    full field solve; a few whole steps timed."""
    import numpy as np
    import oracle
    import pic_inputs as pi

    if workload == "c5":
        wl = pi.c5("cpu", scale=4, z_slab=(220, 228))
        desc = "c5 structure at 64x64x2048 cells, particles in z 220..228 (2 species x 4/cell)"
    elif workload == "c2":
        wl = pi.c2("cpu", scale=4)
        wl.species = [p.select(__import__("torch").nonzero((p.x[2] >= 220) & (p.x[2] < 236)).flatten())
                      for p in wl.species]
        desc = "c2 structure at 32x32x1024 cells, particles in z 220..236"
    else:
        wl = build_workload(workload, "cpu")
        desc = f"{workload} full"
    box = wl.boxes[0]
    g = oracle.make_grid(box.dim, box.n, box.dx, box.dt, box.order)
    sps = [p.numpy() for p in wl.species]
    E = np.ascontiguousarray(wl.E[0].numpy()).copy()
    B = np.ascontiguousarray(wl.B[0].numpy()).copy()
    J = np.zeros_like(E)
    npart = sum(s.x.shape[1] for s in sps)
    steps, t_used = 0, 0.0
    t0 = time.time()
    while steps < 20 and (time.time() - t0) < 12.0:
        oracle.pic_step(g, E, B, J, sps)
        steps += 1
    t_used = time.time() - t0
    return {"value": npart * steps / t_used, "unit": "particle-steps/s", "cores": 1,
            "kind": "oracle",
            "sample": f"{desc}: {npart} particles x {steps} whole steps in {t_used:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c5", choices=["c5", "c2", "c4", "c1", "c3"])
    ap.add_argument("--sort-every", type=int, default=8)
    ap.add_argument("--tile32", type=int, nargs=3, default=(8, 8, 8))
    ap.add_argument("--tile64", type=int, nargs=3, default=(8, 8, 4))
    ap.add_argument("--block", type=int, default=1024)
    ap.add_argument("--block64", type=int, default=512)
    ap.add_argument("--stride", type=int, default=1, help="FP32 lane stride (1: quad-pooled deposit)")
    ap.add_argument("--stride64", type=int, default=4, help="FP64 lane stride")
    ap.add_argument("--chunk", type=int, default=4096)
    ap.add_argument("--wg-per-cu", type=int, default=2)
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 comparison form")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU "
              "slab decomposition is a design, not part of this build.", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2303_12873_amd as pic
    if not os.path.exists(pic.LIB_PATH):
        from paper_2303_12873_amd.build import build
        build()
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)

    t0 = time.time()
    wl = build_workload(args.workload, "cuda")
    torch.cuda.synchronize()
    order = wl.boxes[0].order
    log(f"workload {wl.name}: {wl.np_total} particles, "
        f"{sum(b.ncells for b in wl.boxes)} cells, generated in {time.time() - t0:.1f}s")

    log("FP32 split + batched form")
    r32 = run_form(wl, pic.PIC_FP32_SPLIT, pic.PIC_KERNEL_BATCHED, args.steps, args.warmup,
                   args.sort_every, args.tile32, args.block, args.chunk, args.wg_per_cu, args.stride)
    log(f"  {r32}")
    r64 = None
    if not args.no_fp64:
        log("FP64 plain (tiled) form")
        r64 = run_form(wl, pic.PIC_FP64, pic.PIC_KERNEL_TILED, max(3, args.steps // 4), 1,
                       args.sort_every, args.tile64, args.block64, 0, 0, args.stride64)
        log(f"  {r64}")

    value = r32["np"] * 1e3 / r32["ms_step"]
    ncells = r32["cells"]
    dim3 = all(b.dim == 3 for b in wl.boxes)
    bpp = BYTES_PER_PARTICLE["fp32" if dim3 else "fp32_2d"]
    bytes_launch = r32["np"] * bpp + ncells * BYTES_PER_CELL["fp32"]
    flops_launch = r32["np"] * FLOPS_PER_PARTICLE[order]
    t_adv = r32["ms_advance"] * 1e-3
    gbs = bytes_launch / t_adv / 1e9
    tfl = flops_launch / t_adv / 1e12
    f_hbm, f_alu = gbs / PEAK_HBM_GBS, tfl / PEAK_FP32_TFLOPS
    if f_alu >= f_hbm:
        roof = {"bound": "alu", "achieved": round(tfl, 3), "peak": PEAK_FP32_TFLOPS,
                "unit": "TFLOP/s", "frac": round(f_alu, 4), "traffic": None,
                "hbm_frac": round(f_hbm, 4), "hbm_achieved_GBs": round(gbs, 1)}
    else:
        roof = {"bound": "hbm", "achieved": round(gbs, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": round(f_hbm, 4), "traffic": None, "alu_frac": round(f_alu, 4)}
    roof["kernel"] = "k_tiled<Split, FUSED, persistent> (pic_advance)"
    roof["kernel_ms"] = round(r32["ms_advance"], 4)

    out = {
        "metric": METRIC, "value": value, "unit": "particle-steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": r32["ms_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": wl.name, "cells": ncells, "particles": r32["np"], "order": order,
                   "form": "fp32_split_batched_graph", "sort_every": args.sort_every,
                   "tile": list(args.tile32), "block": args.block, "chunk": args.chunk,
                   "wg_per_cu": args.wg_per_cu, "lane_stride": args.stride},
        "roofline": roof,
        "breakdown_ms": {"advance": r32["ms_advance"], "sort": r32["ms_sort"],
                         "fdtd": r32["ms_fdtd"]},
    }
    if r64 is not None:
        v64 = r64["np"] * 1e3 / r64["ms_step"]
        out["fp64_plain"] = {"value": v64, "ms_per_step": r64["ms_step"],
                             "breakdown_ms": {"advance": r64["ms_advance"], "sort": r64["ms_sort"],
                                              "fdtd": r64["ms_fdtd"]},
                             "tile": list(args.tile64)}
        out["speedup_fp32_batched_vs_fp64_plain"] = value / v64
    if not args.no_cpu:
        log("oracle CPU baseline")
        out["cpu_baseline"] = cpu_baseline(args.workload, order)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
