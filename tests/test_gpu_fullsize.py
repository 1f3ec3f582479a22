"""Parity at full workload sizes, in the launch configuration bench.py times.

The oracle cannot run a billion-particle box, so (1) a random sample of
particles is followed one by one: the oracle gathers E, B for each sampled
particle from the full initial fields, pushes and advances it, and the GPU's
result for the same particle (located through the sort permutation) must
agree; (2) the discrete continuity equation is checked over the whole box on
the GPU in FP64.  Oracle inputs are the generator's arrays, copied to the
host before the GPU touches them.
"""
import numpy as np
import pytest
import torch

import oracle
import pic_inputs as pi
import paper_2303_12873_amd as pic
from pichelp import ensure_built

pytestmark = [pytest.mark.gpu, pytest.mark.slow]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available()
    ensure_built()


def _sampled_parity(wl, precision, kernel, tile, nsample, tol_x, tol_u, tol_cont, block, stride):
    box0 = wl.boxes[0]
    box = pi.Box(box0.dim, box0.n, box0.dt, box0.order, tile, box0.dx)
    g = oracle.make_grid(box.dim, box.n, box.dx, box.dt, box.order)
    rng = np.random.default_rng(17)
    samples = []
    for p in wl.species:
        idx = np.sort(rng.choice(p.np, size=min(nsample, p.np), replace=False))
        it = torch.from_numpy(idx).to(p.x.device)
        samples.append((idx, p.x[:, it].cpu().numpy(), p.u[:, it].cpu().numpy()))
    E0 = np.ascontiguousarray(wl.E[0].cpu().numpy())
    B0 = np.ascontiguousarray(wl.B[0].cpu().numpy())

    # the launch configuration bench.py times (defaults of both forms)
    ctx = pic.pic_init([box], precision, kernel=kernel, block=block, chunk=4096, wg_per_cu=2,
                       lane_stride=stride)
    f = pic.make_fields([box], wl.E, wl.B, precision)
    sp = [pic.make_species(p, precision) for p in wl.species]
    perms = [torch.empty(s.np, dtype=torch.int32, device="cuda") for s in sp]
    pic.pic_sort_tiles(ctx, sp, perm_out=perms)
    rho0 = torch.zeros(box.ncells, dtype=torch.float64, device="cuda")
    pic.pic_deposit_rho(ctx, sp, 0, rho0)
    pic.pic_advance(ctx, f, sp)
    rho1 = torch.zeros_like(rho0)
    pic.pic_deposit_rho(ctx, sp, 0, rho1)
    divj = torch.zeros_like(rho0)
    pic.pic_div_edge(ctx, 0, [f.J[0], f.J[1], f.J[2]], divj)
    pic.pic_check(ctx)
    res = ((rho1 - rho0) / box.dt + divj).abs().max().item()
    scale = divj.abs().max().item()
    assert res <= tol_cont * scale, (res, scale)
    del rho0, rho1, divj

    L = np.array(box.n, dtype=np.float64)
    for s, (p, (idx, x0, u0)) in enumerate(zip(sp, samples)):
        inv = torch.empty_like(perms[s])
        inv[perms[s].long()] = torch.arange(p.np, dtype=torch.int32, device="cuda")
        where = inv[torch.from_numpy(idx).to("cuda")].long()
        ug = p.u[:, where].double().cpu().numpy()
        if p.x is not None:
            xg = p.x[:, where].cpu().numpy()
        else:
            cell = p.cell[where].long().cpu().numpy()
            off = p.off[:, where].double().cpu().numpy()
            xg = np.stack([cell % box.n[0] + off[0], (cell // box.n[0]) % box.n[1] + off[1],
                           cell // (box.n[0] * box.n[1]) + off[2]])
        xo = np.empty_like(x0)
        uo = np.empty_like(u0)
        for k in range(x0.shape[1]):
            Ep, Bp = oracle.gather(g, E0, B0, x0[:, k])
            u = oracle.boris(p.q, p.m, box.dt, Ep, Bp, u0[:, k])
            gam = np.sqrt(1.0 + u @ u)
            for d in range(3):
                xo[d, k] = oracle.wrap(x0[d, k] + box.dt * u[d] / (gam * box.dx[d]), box.n[d])
            uo[:, k] = u
        dx = xg - xo
        dx -= L[:, None] * np.round(dx / L[:, None])
        assert np.max(np.abs(dx)) <= tol_x, np.max(np.abs(dx))
        du = np.linalg.norm(ug - uo) / max(np.linalg.norm(uo), 1e-300)
        assert du <= tol_u, du
    pic.pic_free(ctx)


def test_c5_full_size_split_batched_sampled():
    wl = pi.c5("cuda")
    _sampled_parity(wl, pic.PIC_FP32_SPLIT, pic.PIC_KERNEL_BATCHED, (8, 8, 8), 3000,
                    tol_x=1e-5, tol_u=1e-5, tol_cont=1e-5, block=1024, stride=1)


def test_c5_full_size_fp64_plain_sampled():
    wl = pi.c5("cuda")
    _sampled_parity(wl, pic.PIC_FP64, pic.PIC_KERNEL_TILED, (8, 8, 4), 3000,
                    tol_x=1e-12, tol_u=1e-12, tol_cont=1e-12, block=512, stride=4)


def test_c2_full_size_fp64_tiled_sampled():
    wl = pi.c2("cuda")
    _sampled_parity(wl, pic.PIC_FP64, pic.PIC_KERNEL_TILED, (8, 8, 4), 3000,
                    tol_x=1e-12, tol_u=1e-12, tol_cont=1e-12, block=512, stride=4)
