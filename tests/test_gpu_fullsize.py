"""Parity at full workload sizes, in the launch configurations bench.py
times (``autotune.PICK_FP32`` / ``PICK_FP64`` on the 256x256x2048 box; the
128x128x1024 case in the configuration of bench.py's c2 leg), after the
particles have drifted for a whole sort interval.

The oracle cannot run a billion-particle box, so:
  1. the sort of step 0 runs, then sort_every - 1 whole steps (graph
     replays, no sort), so particles have moved into the staged margin and
     beyond it (the straggler path) as they do before every sort;
  2. the evolved E, B and a random sample of particles (located through the
     step-0 permutation, which no later step changes) are copied to the
     host;
  3. one more step runs on the GPU; the oracle's own particle update
     (orc_particles_step: gather, Boris, advance, deposit, wrap) of the
     sampled particles in the copied fields must give the GPU's positions
     and momenta for the same particles;
  4. the discrete continuity equation of that step is checked over the
     whole box on the GPU in FP64 (rho from pic_deposit_rho before and
     after, div J from pic_div_edge).
"""
import numpy as np
import pytest
import torch

import oracle
import pic_inputs as pi
import paper_2303_12873_amd as pic
from paper_2303_12873_amd.autotune import PICK_FP32, PICK_FP64, Candidate
from pichelp import ensure_built

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

# bench.py's c2 leg
C2_FP64 = Candidate((16, 8, 4), 512, 8192, 2, 4, -1, 8, 0, 0)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available()
    ensure_built()


class _Sample:
    def __init__(self, q, m, x, u, w):
        self.q, self.m = q, m
        self.x = np.ascontiguousarray(x, dtype=np.float64)
        self.u = np.ascontiguousarray(u, dtype=np.float64)
        self.w = np.ascontiguousarray(w, dtype=np.float64)


def _positions(p, where, box):
    if p.x is not None:
        return p.x[:, where].cpu().numpy()
    cell = p.cell[where].long().cpu().numpy()
    off = p.off[:, where].double().cpu().numpy()
    return np.stack([cell % box.n[0] + off[0], (cell // box.n[0]) % box.n[1] + off[1],
                     cell // (box.n[0] * box.n[1]) + off[2]])


def _drifted_parity(wl, precision, kernel, c, nsample, tol_x, tol_u, tol_cont):
    box0 = wl.boxes[0]
    box = pi.Box(box0.dim, box0.n, box0.dt, box0.order, tuple(c.tile), box0.dx)
    g = oracle.make_grid(box.dim, box.n, box.dx, box.dt, box.order)
    rng = np.random.default_rng(17)
    idx = [np.sort(rng.choice(p.np, size=min(nsample, p.np), replace=False)) for p in wl.species]
    ctx = pic.pic_init([box], precision, kernel=kernel, block=c.block, chunk=c.chunk,
                       wg_per_cu=c.wg_per_cu, lane_stride=c.lane_stride,
                       cell_order=c.cell_order, pad=c.pad, margin=c.margin)
    f = pic.make_fields([box], wl.E, wl.B, precision)
    sp = [pic.make_species(p, precision) for p in wl.species]
    wl.species = [p.select(torch.from_numpy(i).to(p.x.device)) for p, i in zip(wl.species, idx)]
    perms = [torch.empty(s.np, dtype=torch.int32, device="cuda") for s in sp]
    pic.pic_sort_tiles(ctx, sp, perm_out=perms)
    where = []
    for s, p in enumerate(sp):
        inv = torch.empty_like(perms[s])
        inv[perms[s].long()] = torch.arange(p.np, dtype=torch.int32, device="cuda")
        where.append(inv[torch.from_numpy(idx[s]).to("cuda")].long())
    del perms
    for k in range(c.sort_every - 1):
        pic.pic_step(ctx, f, sp, sort=False)
    pic.pic_check(ctx)
    # the evolved state the last step of the interval starts from
    E0 = np.ascontiguousarray(f.E.double().cpu().numpy())
    B0 = np.ascontiguousarray(f.B.double().cpu().numpy())
    samples = []
    for s, p in enumerate(sp):
        samples.append(_Sample(p.q, p.m, _positions(p, where[s], box),
                               p.u[:, where[s]].double().cpu().numpy(),
                               p.w[where[s]].double().cpu().numpy()))
    rho0 = torch.zeros(box.ncells, dtype=torch.float64, device="cuda")
    pic.pic_deposit_rho(ctx, sp, 0, rho0)
    pic.pic_step(ctx, f, sp, sort=False)      # the bench's graph of this step
    rho1 = torch.zeros_like(rho0)
    pic.pic_deposit_rho(ctx, sp, 0, rho1)
    divj = torch.zeros_like(rho0)
    pic.pic_div_edge(ctx, 0, [f.J[0], f.J[1], f.J[2]], divj)
    pic.pic_check(ctx)
    res = ((rho1 - rho0) / box.dt + divj).abs().max().item()
    scale = divj.abs().max().item()
    print(f"continuity residual {res:.3e} of max |div J| {scale:.3e}")
    assert res <= tol_cont * scale, (res, scale)
    del rho0, rho1, divj

    # the oracle's particle update of the sampled particles in the copied fields
    J = np.zeros_like(E0)
    oracle.particles_step(g, E0, B0, J, samples)
    del E0, B0, J
    L = np.array(box.n, dtype=np.float64)
    for s, p in enumerate(sp):
        xg = _positions(p, where[s], box)
        ug = p.u[:, where[s]].double().cpu().numpy()
        dx = xg - samples[s].x
        dx -= L[:, None] * np.round(dx / L[:, None])
        print(f"species {s}: max |dx| {np.max(np.abs(dx)):.3e}")
        assert np.max(np.abs(dx)) <= tol_x, np.max(np.abs(dx))
        du = np.linalg.norm(ug - samples[s].u) / max(np.linalg.norm(samples[s].u), 1e-300)
        assert du <= tol_u, du
    pic.pic_free(ctx)
    del f, sp
    torch.cuda.empty_cache()


def test_c5_full_size_split_batched_after_drift():
    wl = pi.c5("cuda")
    _drifted_parity(wl, pic.PIC_FP32_SPLIT, pic.PIC_KERNEL_BATCHED, PICK_FP32, 3000,
                    tol_x=1e-5, tol_u=1e-5, tol_cont=1e-5)


def test_c5_full_size_fp64_plain_after_drift():
    wl = pi.c5("cuda")
    _drifted_parity(wl, pic.PIC_FP64, pic.PIC_KERNEL_TILED, PICK_FP64, 3000,
                    tol_x=1e-12, tol_u=1e-12, tol_cont=1e-12)


def test_c2_full_size_fp64_tiled_after_drift():
    wl = pi.c2("cuda")
    _drifted_parity(wl, pic.PIC_FP64, pic.PIC_KERNEL_TILED, C2_FP64, 3000,
                    tol_x=1e-12, tol_u=1e-12, tol_cont=1e-12)
