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

# Algorithmic work per unit: bytes a particle must move per step (read
# position, u, w; write position, u), bytes per cell of E/B read and J
# written by the particle kernel, and flops per particle (FMA = 2) by shape
# order (gather 12 (n+1)^3, push ~100, Esirkepov deposit).
BYTES_PER_PARTICLE = {"fp64": 104, "fp32": 60, "fp32_2d": 52}
BYTES_PER_CELL = {"fp64": 72, "fp32": 48}
FLOPS_PER_PARTICLE = {1: 550, 2: 1150, 3: 2150}
PEAK_HBM_GBS = 8000.0
# Vector ALU peak the kernels can reach: 256 CUs x 4 SIMDs x 16 lanes x 2
# flops (FMA) x 2.4 GHz = 78.6 TFLOP/s for FP32 without packed-FP32
# instructions (the kernels are built without them) and for FP64.
PEAK_VALU_TFLOPS = 78.6
TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "k_tiled_split_c5_traffic.md")
KERNEL_SOURCES = ("pic_particles.hip", "pic_math.h", "pic_dev.h")


def kernel_source_sha():
    import hashlib
    h = hashlib.sha256()
    for n in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2303_12873_amd", "csrc", n), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def launch_config(tile, block, stride, cell_order, pad, margin):
    return (f"tile={tuple(tile)} block={block} lane_stride={stride} cell_order={cell_order} "
            f"pad={pad} margin={margin}")


def measured_traffic(workload, config):
    """HBM bytes per launch of the particle kernel from the committed
    rocprofv3 counter summary, if it was taken on this workload and launch
    configuration with the current kernel sources; else None."""
    if not os.path.exists(TRAFFIC_SUMMARY):
        return None
    fields = {}
    with open(TRAFFIC_SUMMARY) as f:
        for line in f:
            if ":" in line and line.startswith("- "):
                k, v = line[2:].split(":", 1)
                fields[k.strip()] = v.strip().strip("`")
    if (fields.get("workload") != workload or fields.get("config") != config
            or fields.get("kernel_source_sha256") != kernel_source_sha()):
        return None
    try:
        return int(fields["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


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


def run_form(wl, precision, kernel, steps, warmup, sort_every, tile, block, chunk, wg, stride,
             cell_order=0, pad=0, margin=0):
    import torch
    import paper_2303_12873_amd as pic
    import pic_inputs as pi

    boxes = [pi.Box(b.dim, b.n, b.dt, b.order, tuple(tile) if b.dim == 3 else (tile[0], 1, tile[2]),
                    b.dx) for b in wl.boxes]
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        ctx = pic.pic_init(boxes, precision, stream=stream.cuda_stream, kernel=kernel,
                           block=block, chunk=chunk, wg_per_cu=wg, lane_stride=stride,
                           cell_order=cell_order, pad=pad, margin=margin)
        f = pic.make_fields(boxes, wl.E, wl.B, precision)
        sp = [pic.make_species(p, precision) for p in wl.species]
    torch.cuda.synchronize()
    np_tot = sum(s.np for s in sp)
    # HIP events around the particle kernel inside every step's graph
    pic.pic_set_timing(ctx, True)

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
    kms = []
    for k in range(steps):
        one(k)
        kms.append(pic.pic_kernel_ms(ctx))     # waits for this step's kernel
    ev1.record(stream)
    torch.cuda.synchronize()
    ms_step = ev0.elapsed_time(ev1) / steps
    ms_adv = sum(kms) / len(kms)
    pic.pic_check(ctx)
    pic.pic_set_timing(ctx, False)
    # the sort alone, then the field update alone (breakdown)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
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
                cells=sum(b.ncells for b in boxes), kernel_ms_min=min(kms), kernel_ms_max=max(kms))


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
    ap.add_argument("--cell-order", type=int, default=0,
                    help="FP32 within-tile order without the tuner (-1, 1, 2; 0 = library default)")
    ap.add_argument("--margin", type=int, default=0,
                    help="FP32 staged margin without the tuner (0 where it fits, -1 none)")
    ap.add_argument("--pad", type=int, default=0,
                    help="FP32 LDS row padding without the tuner (-1, 0, 1, 2)")
    ap.add_argument("--no-tune", action="store_true",
                    help="skip the autotuner (use --tile32/--block/--stride and the default order)")
    ap.add_argument("--tune-budget", type=float, default=120.0, help="autotuner time budget (s)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU "
              "slab decomposition is not implemented.", file=sys.stderr)
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

    cell_order = args.cell_order
    tuned = tuned64 = None
    args.sort_every64 = args.sort_every
    args.margin64 = 0
    if not args.no_tune:
        from paper_2303_12873_amd.autotune import tune
        # Tune on the workload itself (a half-size sample ranked the
        # candidates differently).  Each candidate runs its whole sort period
        # (drift included); the picked sort interval is then used by both
        # forms.
        t1 = time.time()
        best, table = tune(wl, pic.PIC_FP32_SPLIT, budget_s=args.tune_budget, cache=None, log=log)
        torch.cuda.empty_cache()
        if best is not None:
            args.tile32, args.block, args.chunk = tuple(best.tile), best.block, best.chunk
            args.wg_per_cu, args.stride, cell_order = best.wg_per_cu, best.lane_stride, best.cell_order
            args.sort_every = best.sort_every
            args.pad = best.pad
            args.margin = best.margin
            tuned = {"picked": best.key(), "candidates": len(table),
                     "seconds": round(time.time() - t1, 1)}
        log(f"  autotuner: {tuned}")
        if not args.no_fp64:
            # the plain FP64 form gets the same search over its own space
            # (non-persistent tiled kernel, 512 threads)
            t1 = time.time()
            best64, table64 = tune(wl, pic.PIC_FP64, budget_s=args.tune_budget, cache=None,
                                   log=log, kernel=pic.PIC_KERNEL_TILED)
            torch.cuda.empty_cache()
            if best64 is not None:
                args.tile64, args.block64 = tuple(best64.tile), best64.block
                args.stride64, args.sort_every64 = best64.lane_stride, best64.sort_every
                args.margin64 = best64.margin
                tuned64 = {"picked": best64.key(), "candidates": len(table64),
                           "seconds": round(time.time() - t1, 1)}
            log(f"  autotuner (FP64 plain): {tuned64}")
    log("FP32 split + batched form")
    r32 = run_form(wl, pic.PIC_FP32_SPLIT, pic.PIC_KERNEL_BATCHED, args.steps, args.warmup,
                   args.sort_every, args.tile32, args.block, args.chunk, args.wg_per_cu, args.stride,
                   cell_order, args.pad, args.margin)
    log(f"  {r32}")
    r64 = None
    if not args.no_fp64:
        log("FP64 plain (tiled) form")
        r64 = run_form(wl, pic.PIC_FP64, pic.PIC_KERNEL_TILED, args.steps, args.warmup,
                       args.sort_every64, args.tile64, args.block64, 0, 0, args.stride64,
                       -1, 0, args.margin64)
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
    f_hbm, f_alu = gbs / PEAK_HBM_GBS, tfl / PEAK_VALU_TFLOPS
    traffic = measured_traffic(wl.name, launch_config(args.tile32, args.block, args.stride,
                                                       cell_order, args.pad, args.margin))
    if f_alu >= f_hbm:
        roof = {"bound": "alu", "achieved": round(tfl, 3), "peak": PEAK_VALU_TFLOPS,
                "unit": "TFLOP/s", "frac": round(f_alu, 4), "traffic": traffic,
                "hbm_frac": round(f_hbm, 4), "hbm_achieved_GBs": round(gbs, 1)}
    else:
        roof = {"bound": "hbm", "achieved": round(gbs, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": round(f_hbm, 4), "traffic": traffic, "alu_frac": round(f_alu, 4)}
    roof["kernel"] = "k_tiled<Split, FUSED, persistent> (particle part of each step's graph)"
    roof["kernel_ms"] = round(r32["ms_advance"], 4)
    roof["algorithmic_bytes_per_launch"] = bytes_launch
    roof["algorithmic_flops_per_launch"] = flops_launch

    out = {
        "metric": METRIC, "value": value, "unit": "particle-steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": r32["ms_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": wl.name, "cells": ncells, "particles": r32["np"], "order": order,
                   "form": "fp32_split_batched_graph", "sort_every": args.sort_every,
                   "tile": list(args.tile32), "block": args.block, "chunk": args.chunk,
                   "wg_per_cu": args.wg_per_cu, "lane_stride": args.stride,
                   "cell_order": cell_order, "pad": args.pad, "margin": args.margin,
                   "autotuned": tuned},
        "roofline": roof,
        "breakdown_ms": {"advance": r32["ms_advance"], "sort": r32["ms_sort"],
                         "fdtd": r32["ms_fdtd"]},
    }
    if r64 is not None:
        v64 = r64["np"] * 1e3 / r64["ms_step"]
        out["fp64_plain"] = {"value": v64, "ms_per_step": r64["ms_step"],
                             "breakdown_ms": {"advance": r64["ms_advance"], "sort": r64["ms_sort"],
                                              "fdtd": r64["ms_fdtd"]},
                             "tile": list(args.tile64), "block": args.block64,
                             "lane_stride": args.stride64, "sort_every": args.sort_every64,
                             "margin": args.margin64, "autotuned": tuned64}
        out["speedup_fp32_batched_vs_fp64_plain"] = value / v64
    if not args.no_cpu:
        log("oracle CPU baseline")
        out["cpu_baseline"] = cpu_baseline(args.workload, order)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
