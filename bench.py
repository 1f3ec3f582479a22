"""Benchmark of the PIC hot path on one MI355X.

One step = the whole hot path over the workload: per-tile sort (every
``sort_every`` steps, amortised), fused gather + Boris push + Esirkepov
deposit, and the Yee update, issued as one captured HIP graph launch.  The
headline ``value`` is particle-steps/s of the FP32 split-precision batched
form on the largest single-GPU case; the plain FP64 form runs on the same
inputs beside it.

Headline workload: 256x256x2048 cells, electrons and ions (mass ratio 1836)
at 4 each per cell behind a 120-cell vacuum with a 100-cell density ramp,
order-3 shapes, a0 = 4 Gaussian laser; inputs are generated on the device
from seeded generators (``pic_inputs``).  Both forms run in the launch
configurations the autotuner picks on that box (``autotune.PICK_FP32`` /
``PICK_FP64``; ``--tune`` re-runs the tuner).

Extra keys of the JSON line (each its own leg, all on synthetic inputs):
  error      FP32 split vs FP64 plain in lockstep on the headline inputs:
             per-step relative L2 of E, B, J and the relative difference of
             the total (field + kinetic) energy, plus each form's energy
             change since step 0;
  laser      a second FP32 window, after the laser's centroid has travelled
             to the plasma ramp (steps 100..148);
  c2_fp64    128x128x1024, 2 electrons/cell, order 2, FP64 plain: the
             particle kernel against the HBM roofline (the case whose
             algorithmic bytes are the largest share of its work);
  c4         64 2D boxes + one 3D box with lognormal tile counts: FP32
             batched vs FP64 plain;
  cpu_baseline  the FP64 oracle's particle update on host cores.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import platform
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
BYTES_PER_PARTICLE = {"fp64": 104, "fp32": 60, "fp32_2d": 52, "fp64_2d": 88}
BYTES_PER_CELL = {"fp64": 72, "fp32": 48}
FLOPS_PER_PARTICLE = {1: 550, 2: 1150, 3: 2150}
PEAK_HBM_GBS = 8000.0
# Vector ALU peak the kernels can reach: 256 CUs x 4 SIMDs x 16 lanes x 2
# flops (FMA) x 2.4 GHz = 78.6 TFLOP/s for FP32 without packed-FP32
# instructions (the kernels are built without them) and for FP64.
PEAK_VALU_TFLOPS = 78.6
TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "k_tiled_split_c5_traffic.md")
# the particle kernel and the host code that lays out its LDS tiles
KERNEL_SOURCES = ("pic_particles.hip", "pic_math.h", "pic_dev.h", "libpic.hip")


def kernel_source_sha():
    import hashlib
    h = hashlib.sha256()
    for n in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2303_12873_amd", "csrc", n), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def launch_config(c):
    return (f"tile={tuple(c.tile)} block={c.block} lane_stride={c.lane_stride} "
            f"cell_order={c.cell_order} pad={c.pad} margin={c.margin}")


def measured_traffic(workload, config, path=TRAFFIC_SUMMARY):
    """HBM bytes per launch of the particle kernel from a committed
    rocprofv3 counter summary, if it was taken on this workload and launch
    configuration with the current kernel sources; else None."""
    if not os.path.exists(path):
        return None
    fields = {}
    with open(path) as f:
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


def _boxes(wl, tile):
    import pic_inputs as pi
    return [pi.Box(b.dim, b.n, b.dt, b.order, tuple(tile) if b.dim == 3 else (tile[0], 1, tile[2]),
                   b.dx) for b in wl.boxes]


class Form:
    """One precision form of a workload on the device: context (bound to a
    stream of its own), fields and species, in launch configuration ``c``."""

    def __init__(self, wl, precision, kernel, c):
        import torch
        import paper_2303_12873_amd as pic
        self.pic, self.torch = pic, torch
        self.c = c
        self.boxes = _boxes(wl, c.tile)
        self.stream = torch.cuda.Stream()
        with torch.cuda.stream(self.stream):
            self.ctx = pic.pic_init(self.boxes, precision, stream=self.stream.cuda_stream,
                                    kernel=kernel, block=c.block, chunk=c.chunk,
                                    wg_per_cu=c.wg_per_cu, lane_stride=c.lane_stride,
                                    cell_order=c.cell_order, pad=c.pad, margin=c.margin)
            self.f = pic.make_fields(self.boxes, wl.E, wl.B, precision)
            self.sp = [pic.make_species(p, precision) for p in wl.species]
        torch.cuda.synchronize()
        self.k = 0
        self.np = sum(s.np for s in self.sp)
        self.cells = sum(b.ncells for b in self.boxes)

    def step(self):
        self.pic.pic_step(self.ctx, self.f, self.sp, sort=(self.k % self.c.sort_every == 0))
        self.k += 1

    def energy(self):
        out = self.torch.zeros(2 + len(self.sp), dtype=self.torch.float64, device="cuda")
        tot = 0.0
        for b in range(len(self.boxes)):
            self.pic.pic_energy(self.ctx, self.f, self.sp, b, out)
            self.torch.cuda.synchronize()
            tot += float(out.sum())
        return tot

    def timed(self, steps):
        """Time `steps` graph replays; per-step particle-kernel time from the
        library's device clock stamps."""
        torch, pic = self.torch, self.pic
        pic.pic_set_timing(self.ctx, True)
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        ev0.record(self.stream)
        kms = []
        for _ in range(steps):
            self.step()
            kms.append(pic.pic_kernel_ms(self.ctx))
        ev1.record(self.stream)
        torch.cuda.synchronize()
        pic.pic_check(self.ctx)
        pic.pic_set_timing(self.ctx, False)
        return ev0.elapsed_time(ev1) / steps, kms

    def breakdown(self):
        """The sort alone, then the field update alone (one call each)."""
        torch, pic = self.torch, self.pic
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(self.stream)
        pic.pic_sort_tiles(self.ctx, self.sp)
        e1.record(self.stream)
        torch.cuda.synchronize()
        ms_sort = e0.elapsed_time(e1)
        e0.record(self.stream)
        pic.pic_fdtd_step(self.ctx, self.f)
        e1.record(self.stream)
        torch.cuda.synchronize()
        pic.pic_check(self.ctx)
        return ms_sort, e0.elapsed_time(e1)

    def free(self):
        self.pic.pic_free(self.ctx)
        del self.f, self.sp
        self.torch.cuda.empty_cache()


def run_form(wl, precision, kernel, c, steps, warmup):
    fm = Form(wl, precision, kernel, c)
    t0 = time.time()
    for _ in range(warmup):
        fm.step()
    fm.torch.cuda.synchronize()
    log(f"  warmup {warmup} steps {time.time() - t0:.2f}s")
    ms_step, kms = fm.timed(steps)
    ms_sort, ms_fdtd = fm.breakdown()
    out = dict(np=fm.np, cells=fm.cells, ms_step=ms_step, ms_advance=sum(kms) / len(kms),
               ms_sort=ms_sort, ms_fdtd=ms_fdtd, kernel_ms_min=min(kms), kernel_ms_max=max(kms),
               kernel_ms_steps=[round(x, 2) for x in kms])
    fm.free()
    return out


def roofline(np_tot, ncells, order, dim3, prec, kernel_ms, traffic=None, bound=None):
    """Algorithmic bytes and flops of one particle-kernel launch over its
    measured duration, against the HBM and vector-ALU peaks."""
    key = prec if dim3 else prec + "_2d"
    bytes_launch = np_tot * BYTES_PER_PARTICLE[key] + ncells * BYTES_PER_CELL[prec]
    flops_launch = np_tot * FLOPS_PER_PARTICLE[order]
    t = kernel_ms * 1e-3
    gbs = bytes_launch / t / 1e9
    tfl = flops_launch / t / 1e12
    f_hbm, f_alu = gbs / PEAK_HBM_GBS, tfl / PEAK_VALU_TFLOPS
    if bound is None:
        bound = "alu" if f_alu >= f_hbm else "hbm"
    if bound == "alu":
        r = {"bound": "alu", "achieved": round(tfl, 3), "peak": PEAK_VALU_TFLOPS,
             "unit": "TFLOP/s", "frac": round(f_alu, 4), "traffic": traffic,
             "hbm_frac": round(f_hbm, 4), "hbm_achieved_GBs": round(gbs, 1)}
    else:
        r = {"bound": "hbm", "achieved": round(gbs, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
             "frac": round(f_hbm, 4), "traffic": traffic, "alu_frac": round(f_alu, 4),
             "alu_achieved_TFLOPs": round(tfl, 3)}
    r["kernel_ms"] = round(kernel_ms, 4)
    r["algorithmic_bytes_per_launch"] = bytes_launch
    r["algorithmic_flops_per_launch"] = flops_launch
    return r


# Yee step per cell: algorithmic = read E, B, J once and write E, B once
# (FP64: 120 B; split: FP32 E/B, FP64 J: 72 B); as run, three streaming
# passes (B half: read E, B, write B; E: read E, B, J, write E; B half).
FDTD_BYTES_PER_CELL = {"fp64": 120, "fp32": 72}
FDTD_PASS_BYTES_PER_CELL = {"fp64": 72 + 96 + 72, "fp32": 36 + 60 + 36}


def fdtd_roofline(ncells, prec, ms):
    """HBM fractions of one pic_fdtd_step over its measured duration."""
    t = ms * 1e-3
    alg = ncells * FDTD_BYTES_PER_CELL[prec]
    run = ncells * FDTD_PASS_BYTES_PER_CELL[prec]
    return {"ms": round(ms, 4), "algorithmic_bytes": alg,
            "hbm_frac": round(alg / t / 1e9 / PEAK_HBM_GBS, 4),
            "bytes_three_passes": run,
            "hbm_frac_three_passes": round(run / t / 1e9 / PEAK_HBM_GBS, 4)}


# ------------------------------------------------------------------ legs

def leg_error(wl, c32, c64, steps):
    """FP32 split vs FP64 plain in lockstep on the same inputs."""
    import paper_2303_12873_amd as pic
    import torch
    a = Form(wl, pic.PIC_FP32_SPLIT, pic.PIC_KERNEL_BATCHED, c32)
    b = Form(wl, pic.PIC_FP64, pic.PIC_KERNEL_TILED, c64)
    w32_0, w64_0 = a.energy(), b.energy()

    def rel(x, y):
        return float((x.double() - y).norm() / y.norm().clamp_min(1e-300))

    rows = []
    for k in range(steps):
        a.step()
        b.step()
        torch.cuda.synchronize()
        w32, w64 = a.energy(), b.energy()
        rows.append({"step": k + 1, "E": rel(a.f.E, b.f.E), "B": rel(a.f.B, b.f.B),
                     "J": rel(a.f.J, b.f.J), "energy": abs(w32 - w64) / w64,
                     "energy_change_fp32": (w32 - w32_0) / w32_0,
                     "energy_change_fp64": (w64 - w64_0) / w64_0})
        log("  step %2d  rel E %.2e  B %.2e  J %.2e  energy %.2e" %
            (k + 1, rows[-1]["E"], rows[-1]["B"], rows[-1]["J"], rows[-1]["energy"]))
    pic.pic_check(a.ctx)
    pic.pic_check(b.ctx)
    a.free()
    b.free()
    return {"steps": steps, "per_step": [{k: (round(v, 4) if k == "step" else float(f"{v:.3e}"))
                                          for k, v in r.items()} for r in rows],
            "max": {q: max(r[q] for r in rows) for q in ("E", "B", "J", "energy")}}


def leg_laser(wl, c32, start, steps):
    """FP32 batched after `start` steps (the laser at the density ramp)."""
    import paper_2303_12873_amd as pic
    fm = Form(wl, pic.PIC_FP32_SPLIT, pic.PIC_KERNEL_BATCHED, c32)
    t0 = time.time()
    for k in range(start):
        fm.step()
        if (k + 1) % 25 == 0:
            fm.torch.cuda.synchronize()
            log(f"  laser leg: {k + 1} steps in {time.time() - t0:.1f}s")
    ms_step, kms = fm.timed(steps)
    v = fm.np * 1e3 / ms_step
    fm.free()
    return {"steps": [start, start + steps], "value": v, "ms_per_step": ms_step,
            "kernel_ms": sum(kms) / len(kms), "kernel_ms_min": min(kms), "kernel_ms_max": max(kms),
            "kernel_ms_per_step": [round(x, 2) for x in kms]}


def _c2_config():
    from paper_2303_12873_amd.autotune import Candidate
    # the fastest of a sweep over tiles 4x4x4 .. 16x8x4 (larger ones exceed
    # the LDS budget in FP64), 256 / 512 threads, tiled and batched kernels,
    # lane stride 4 / tile order and 1 / rank-major, sort every 8 or 16 steps
    return Candidate((16, 8, 4), 512, 8192, 2, 4, -1, 8, 0, 0)


def leg_c2(steps, warmup):
    import paper_2303_12873_amd as pic
    import pic_inputs as pi
    from paper_2303_12873_amd.autotune import Candidate
    import torch
    wl = pi.c2("cuda")
    torch.cuda.synchronize()
    c64 = _c2_config()
    r = run_form(wl, pic.PIC_FP64, pic.PIC_KERNEL_TILED, c64, steps, warmup)
    roof = roofline(r["np"], r["cells"], 2, True, "fp64", r["ms_advance"], bound="hbm",
                    traffic=measured_traffic(wl.name, launch_config(c64),
                                             os.path.join(ROOT, "profiles",
                                                          "k_tiled_fp64_c2_traffic.md")))
    roof["kernel"] = "k_tiled<F64, FUSED, one workgroup per tile> + k_strag"
    del wl
    torch.cuda.empty_cache()
    return {"workload": "c2_lwfa_128x128x1024_ppc2_order2", "particles": r["np"],
            "cells": r["cells"], "value": r["np"] * 1e3 / r["ms_step"],
            "ms_per_step": r["ms_step"], "config": launch_config(c64),
            "breakdown_ms": {"advance": r["ms_advance"], "sort": r["ms_sort"],
                             "fdtd": r["ms_fdtd"]},
            "roofline": roof}


def leg_c4(steps, warmup):
    import paper_2303_12873_amd as pic
    import pic_inputs as pi
    from paper_2303_12873_amd.autotune import Candidate
    import torch
    wl = pi.c4("cuda")
    torch.cuda.synchronize()
    c32 = Candidate((8, 8, 8), 1024, 4096, 2, 4, -1, 16, 0, 0)
    c64 = Candidate((8, 8, 8), 512, 4096, 2, 4, -1, 16, 0, 0)
    r32 = run_form(wl, pic.PIC_FP32_SPLIT, pic.PIC_KERNEL_BATCHED, c32, steps, warmup)
    r64 = run_form(wl, pic.PIC_FP64, pic.PIC_KERNEL_TILED, c64, steps, warmup)
    v32, v64 = r32["np"] * 1e3 / r32["ms_step"], r64["np"] * 1e3 / r64["ms_step"]
    del wl
    torch.cuda.empty_cache()
    return {"workload": "c4_batched_64x2d_plus_256cube_lognormal", "particles": r32["np"],
            "fp32_batched": {"value": v32, "ms_per_step": r32["ms_step"],
                             "advance_ms": r32["ms_advance"], "config": launch_config(c32)},
            "fp64_plain": {"value": v64, "ms_per_step": r64["ms_step"],
                           "advance_ms": r64["ms_advance"], "config": launch_config(c64)},
            "speedup": v32 / v64}


# ------------------------------------------------------------------ CPU baseline

def _oracle_slab(args):
    """One single-threaded oracle process: the particle update (gather,
    push, deposit, wrap; no field solve) of the particles of the 64x64x2048
    copy of the headline box that lie in cell layers [z0, z0 + 8), for
    `steps` timed steps after one untimed one.  Returns (particle-steps,
    seconds)."""
    z0, steps = args
    import numpy as np
    import oracle
    import pic_inputs as pi
    wl = pi.c5("cpu", scale=4, z_slab=(z0, z0 + 8))
    box = wl.boxes[0]
    g = oracle.make_grid(box.dim, box.n, box.dx, box.dt, box.order)
    sps = [p.numpy() for p in wl.species]
    E = np.ascontiguousarray(wl.E[0].numpy()).copy()
    B = np.ascontiguousarray(wl.B[0].numpy()).copy()
    J = np.zeros_like(E)
    npart = sum(s.x.shape[1] for s in sps)
    oracle.particles_step(g, E, B, J, sps)      # untimed: first touch of the arrays
    t0 = time.time()
    for _ in range(steps):
        oracle.particles_step(g, E, B, J, sps)
    return npart * steps, time.time() - t0


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def cpu_baseline(single_steps=3, multi_steps=2):
    """The FP64 oracle's particle update (what the GPU's particle kernel
    computes), timed on host cores: one process, then one single-threaded
    process per usable core (at most 16) on disjoint 8-layer slabs."""
    import multiprocessing as mp
    ps, sec = _oracle_slab((220, single_steps))
    v1 = ps / sec
    nproc = os.cpu_count() or 1
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = nproc
    workers = max(1, min(16, usable))
    ctx = mp.get_context("spawn")
    t0 = time.time()
    with ctx.Pool(workers) as pool:
        res = pool.map(_oracle_slab, [(220 + 8 * i, multi_steps) for i in range(workers)])
    wall = time.time() - t0
    tot_ps = sum(r[0] for r in res)
    slowest = max(r[1] for r in res)
    return {"value": v1, "unit": "particle-steps/s", "cores": 1, "kind": "oracle",
            "sample": (f"particle update only (gather, Boris, advance, Esirkepov, wrap) of the "
                       f"particles in cell layers z 220..228 of a 64x64x2048 copy of the "
                       f"headline box (2 species x 4/cell, order 3, laser fields): "
                       f"{ps} particle-steps in {sec:.1f} s"),
            "all_cores": {"value": tot_ps / slowest, "cores": workers,
                          "processes": workers, "wall_s_incl_setup": round(wall, 1),
                          "sample": f"{workers} single-threaded processes, disjoint 8-layer slabs "
                                    f"from z 220, {multi_steps} steps each"},
            "host": {"nproc": nproc, "usable_cpus": usable, "cpu_model": cpu_model()}}


# ------------------------------------------------------------------ main

def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--tune", action="store_true", help="re-run the autotuner on the headline box")
    ap.add_argument("--tune-budget", type=float, default=120.0)
    ap.add_argument("--legs", default="error,laser,c2,c4,cpu",
                    help="extra legs (comma list of error, laser, c2, c4, cpu; '' for none)")
    ap.add_argument("--error-steps", type=int, default=10)
    ap.add_argument("--laser-start", type=int, default=100)
    ap.add_argument("--laser-steps", type=int, default=48)
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 comparison form")
    ap.add_argument("--tile32", type=int, nargs=3, default=None)
    ap.add_argument("--sort-every", type=int, default=None)
    ap.add_argument("--cell-order", type=int, default=None)
    ap.add_argument("--stride", type=int, default=None, help="FP32 lane stride override")
    ap.add_argument("--pad", type=int, default=None, help="FP32 LDS row padding override")
    ap.add_argument("--cell-order64", type=int, default=None)
    ap.add_argument("--stride64", type=int, default=None)
    ap.add_argument("--sort-every64", type=int, default=None)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}): the library's "
              "slab decomposition runs inside one device, and exchanges between GPUs are not "
              "part of it.", file=sys.stderr)
        sys.exit(2)
    legs = [x for x in args.legs.split(",") if x]

    import dataclasses
    import torch
    import paper_2303_12873_amd as pic
    import pic_inputs as pi
    from paper_2303_12873_amd.autotune import PICK_FP32, PICK_FP64
    if not os.path.exists(pic.LIB_PATH):
        raise SystemExit(f"{pic.LIB_PATH} is not built: run python -m paper_2303_12873_amd.build")
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)

    c32, c64 = PICK_FP32, PICK_FP64
    if args.tile32:
        c32 = dataclasses.replace(c32, tile=tuple(args.tile32))
    if args.sort_every:
        c32 = dataclasses.replace(c32, sort_every=args.sort_every)
    if args.cell_order is not None:
        c32 = dataclasses.replace(c32, cell_order=args.cell_order)
    if args.stride is not None:
        c32 = dataclasses.replace(c32, lane_stride=args.stride)
    if args.pad is not None:
        c32 = dataclasses.replace(c32, pad=args.pad)
    if args.cell_order64 is not None:
        c64 = dataclasses.replace(c64, cell_order=args.cell_order64)
    if args.stride64 is not None:
        c64 = dataclasses.replace(c64, lane_stride=args.stride64)
    if args.sort_every64 is not None:
        c64 = dataclasses.replace(c64, sort_every=args.sort_every64)
    t0 = time.time()
    wl = pi.c5("cuda")
    torch.cuda.synchronize()
    order = wl.boxes[0].order
    log(f"workload {wl.name}: {wl.np_total} particles, "
        f"{sum(b.ncells for b in wl.boxes)} cells, generated in {time.time() - t0:.1f}s")

    tuned = tuned64 = None
    if args.tune:
        from paper_2303_12873_amd.autotune import tune
        t1 = time.time()
        best, table = tune(wl, pic.PIC_FP32_SPLIT, budget_s=args.tune_budget, cache=None, log=log)
        if best is not None:
            c32 = best
            tuned = {"picked": best.key(), "candidates": len(table),
                     "seconds": round(time.time() - t1, 1)}
        torch.cuda.empty_cache()
        if not args.no_fp64:
            t1 = time.time()
            best64, table64 = tune(wl, pic.PIC_FP64, budget_s=args.tune_budget, cache=None,
                                   log=log, kernel=pic.PIC_KERNEL_TILED)
            if best64 is not None:
                c64 = best64
                tuned64 = {"picked": best64.key(), "candidates": len(table64),
                           "seconds": round(time.time() - t1, 1)}
            torch.cuda.empty_cache()
    log(f"FP32 split + batched form: {c32.key()}")
    r32 = run_form(wl, pic.PIC_FP32_SPLIT, pic.PIC_KERNEL_BATCHED, c32, args.steps, args.warmup)
    log(f"  {r32}")
    r64 = None
    if not args.no_fp64:
        log(f"FP64 plain (tiled) form: {c64.key()}")
        r64 = run_form(wl, pic.PIC_FP64, pic.PIC_KERNEL_TILED, c64, args.steps, args.warmup)
        log(f"  {r64}")

    value = r32["np"] * 1e3 / r32["ms_step"]
    ncells = r32["cells"]
    roof = roofline(r32["np"], ncells, order, True, "fp32", r32["ms_advance"],
                    traffic=measured_traffic(wl.name, launch_config(c32)))
    roof["kernel"] = ("k_tiled<Split, FUSED, persistent> + k_strag (particle part of each "
                      "step's graph)")

    out = {
        "metric": METRIC, "value": value, "unit": "particle-steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": r32["ms_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": wl.name, "cells": ncells, "particles": r32["np"], "order": order,
                   "form": "fp32_split_batched_graph", "sort_every": c32.sort_every,
                   "tile": list(c32.tile), "block": c32.block, "chunk": c32.chunk,
                   "wg_per_cu": c32.wg_per_cu, "lane_stride": c32.lane_stride,
                   "cell_order": c32.cell_order, "pad": c32.pad, "margin": c32.margin,
                   "autotuned": tuned},
        "roofline": roof,
        "breakdown_ms": {"advance": r32["ms_advance"], "advance_min": r32["kernel_ms_min"],
                         "advance_max": r32["kernel_ms_max"], "sort": r32["ms_sort"],
                         "fdtd": r32["ms_fdtd"], "advance_per_step": r32["kernel_ms_steps"]},
        "fdtd_roofline": fdtd_roofline(ncells, "fp32", r32["ms_fdtd"]),
    }
    if r64 is not None:
        v64 = r64["np"] * 1e3 / r64["ms_step"]
        out["fp64_plain"] = {"value": v64, "ms_per_step": r64["ms_step"],
                             "breakdown_ms": {"advance": r64["ms_advance"], "sort": r64["ms_sort"],
                                              "fdtd": r64["ms_fdtd"],
                                              "advance_per_step": r64["kernel_ms_steps"]},
                             "config": launch_config(c64), "sort_every": c64.sort_every,
                             "autotuned": tuned64,
                             "fdtd_roofline": fdtd_roofline(r64["cells"], "fp64", r64["ms_fdtd"])}
        out["speedup_fp32_batched_vs_fp64_plain"] = value / v64
    torch.cuda.empty_cache()
    if "error" in legs and not args.no_fp64:
        log(f"error leg: FP32 split vs FP64 plain, {args.error_steps} steps in lockstep")
        out["error"] = leg_error(wl, c32, c64, args.error_steps)
    if "laser" in legs:
        log(f"laser leg: FP32 window steps {args.laser_start}..{args.laser_start + args.laser_steps}")
        out["laser"] = leg_laser(wl, c32, args.laser_start, args.laser_steps)
    del wl
    torch.cuda.empty_cache()
    if "c2" in legs:
        log("c2 leg: FP64 plain, order 2")
        out["c2_fp64"] = leg_c2(args.steps, args.warmup)
    if "c4" in legs:
        log("c4 leg: batched boxes")
        out["c4"] = leg_c4(max(args.steps // 2, 4), args.warmup)
    if "cpu" in legs:
        log("oracle CPU baseline")
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
