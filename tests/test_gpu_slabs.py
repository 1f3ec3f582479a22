"""One periodic box decomposed into z-slabs held as the boxes of one
context (guard-layer fill, J guard reduction, particle migration), against
the oracle's undivided box: the same fields, currents and particles after
several steps, in both precisions."""
import numpy as np
import pytest
import torch

import oracle
import pic_inputs as pi
from pichelp import ensure_built, node_max_rel, rel_l2
import paper_2303_12873_amd as pic

pytestmark = pytest.mark.gpu

G = 3


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    ensure_built()


def _split(wl, nz_slabs):
    """Slab boxes, their fields (interior from the global arrays, guards
    zero until pic_slab_fill_guards) and particles (z shifted to the slab's
    frame)."""
    box = wl.boxes[0]
    nx, ny, nz = box.n
    assert sum(nz_slabs) == nz
    boxes, Es, Bs, sps = [], [], [], []
    z0 = 0
    for s, nzs in enumerate(nz_slabs):
        b = pi.Box(box.dim, (nx, ny, nzs + 2 * G), box.dt, box.order, box.tile, box.dx)
        boxes.append(b)
        for F, out in ((wl.E[0], Es), (wl.B[0], Bs)):
            f = torch.zeros((3, nzs + 2 * G, ny, nx), dtype=torch.float64)
            f[:, G:G + nzs] = F.reshape(3, nz, ny, nx)[:, z0:z0 + nzs]
            out.append(f.reshape(3, -1))
        for p in wl.species:
            sel = torch.nonzero((p.x[2] >= z0) & (p.x[2] < z0 + nzs)).flatten()
            x = p.x[:, sel].clone()
            x[2] += G - z0
            sps.append((s, pi.particles_from_positions(b, x.numpy(), p.u[:, sel].numpy(),
                                                       p.w[sel].numpy(), p.q, p.m, box_index=s)))
        z0 += nzs
    return boxes, Es, Bs, sps


def _gather_fields(t, boxes, nz_slabs, nx, ny):
    out = []
    base = 0
    for b, nzs in zip(boxes, nz_slabs):
        v = t[:, base:base + b.ncells].reshape(3, nzs + 2 * G, ny, nx)[:, G:G + nzs]
        out.append(v)
        base += b.ncells
    return torch.cat(out, dim=1).reshape(3, -1).double().cpu().numpy()


def _global_particles(sp_dev, boxes, z0s, nkind):
    xs, us, ws = [[] for _ in range(nkind)], [[] for _ in range(nkind)], [[] for _ in range(nkind)]
    for i, s in enumerate(sp_dev):
        slab = i // nkind
        b = boxes[slab]
        n = s.np
        if s.x is not None:
            x = s.x[:, :n].double().cpu().numpy().copy()
        else:
            cell = s.cell[:n].long().cpu().numpy()
            off = s.off[:, :n].double().cpu().numpy()
            x = np.stack([cell % b.n[0] + off[0], (cell // b.n[0]) % b.n[1] + off[1],
                          cell // (b.n[0] * b.n[1]) + off[2]])
        x[2] += z0s[slab] - G
        xs[i % nkind].append(x)
        us[i % nkind].append(s.u[:, :n].double().cpu().numpy())
        ws[i % nkind].append(s.w[:n].double().cpu().numpy())
    return ([np.concatenate(x, axis=1) for x in xs], [np.concatenate(u, axis=1) for u in us],
            [np.concatenate(w) for w in ws])


@pytest.mark.parametrize("prec,kernel,tol", ((pic.PIC_FP64, pic.PIC_KERNEL_TILED, 1e-12),
                                             (pic.PIC_FP32_SPLIT, pic.PIC_KERNEL_BATCHED, 1e-5)))
@pytest.mark.parametrize("order", (1, 3))
@pytest.mark.parametrize("dim", (3, 2))
def test_slabs_equal_undivided_box(dim, order, prec, kernel, tol):
    nz_slabs = (8, 7, 9, 8)
    n = (12, 10, sum(nz_slabs))
    wl = pi.uniform_box(n, 3, 0.05, 0.15, order, 7300 + order + 10 * dim, "cpu", tile=(4, 4, 4),
                        fields="fourier", dim=dim, species=("e", "i"))
    # distinct FP32-exact weights label the particles (matched by weight)
    for p in wl.species:
        p.w = 2.0 ** -6 * (1.0 + torch.arange(p.np, dtype=torch.float64) * 2.0 ** -20)
    box = wl.boxes[0]
    nx, ny = box.n[0], box.n[1]
    steps = 6
    # oracle on the undivided box
    g = oracle.make_grid(box.dim, box.n, box.dx, box.dt, box.order)
    sps = [p.numpy() for p in wl.species]
    Eo = wl.E[0].numpy().copy()
    Bo = wl.B[0].numpy().copy()
    Jo = np.zeros_like(Eo)
    for _ in range(steps):
        oracle.pic_step(g, Eo, Bo, Jo, sps)
    # the slabs
    boxes, Es, Bs, sl = _split(wl, nz_slabs)
    nkind = len(wl.species)
    ctx = pic.pic_init(boxes, prec, kernel=kernel)
    f = pic.make_fields(boxes, Es, Bs, prec)
    sp = [pic.make_species(p, prec, capacity=2 * p.np + 64) for _, p in sl]
    z0s = np.cumsum((0,) + nz_slabs[:-1])
    moved = 0
    for _ in range(steps):
        pic.pic_slab_fill_guards(ctx, f, G)
        pic.pic_sort_tiles(ctx, sp)
        pic.pic_advance(ctx, f, sp)
        pic.pic_slab_reduce_j(ctx, f, G)
        pic.pic_fdtd_step(ctx, f)
        before = [s.np for s in sp]
        pic.pic_slab_migrate(ctx, sp, G)
        moved += sum(abs(a - s.np) for a, s in zip(before, sp))
        pic.pic_check(ctx)
    assert moved > 0            # particles did cross slab faces
    E = _gather_fields(f.E, boxes, nz_slabs, nx, ny)
    B = _gather_fields(f.B, boxes, nz_slabs, nx, ny)
    J = _gather_fields(f.J, boxes, nz_slabs, nx, ny)
    for a, b, name in ((E, Eo, "E"), (B, Bo, "B"), (J, Jo, "J")):
        assert rel_l2(a, b) <= tol, (name, rel_l2(a, b))
        assert node_max_rel(a, b) <= tol, (name, node_max_rel(a, b))
    xs, us, ws = _global_particles(sp, boxes, z0s, nkind)
    L = np.array(box.n, dtype=np.float64)[:, None]
    for k in range(nkind):
        assert xs[k].shape[1] == sps[k].x.shape[1]
        og, oo = np.argsort(ws[k], kind="stable"), np.argsort(sps[k].w, kind="stable")
        np.testing.assert_array_equal(ws[k][og], sps[k].w[oo])     # every particle once
        d = xs[k][:, og] - sps[k].x[:, oo]
        d -= L * np.round(d / L)
        if dim == 2:
            d[1] = 0.0
        assert np.max(np.abs(d)) <= (tol if prec == pic.PIC_FP64 else 1e-5) * max(box.n), np.max(np.abs(d))
        assert rel_l2(us[k][:, og], sps[k].u[:, oo]) <= tol
    pic.pic_free(ctx)


def test_slab_arguments_checked():
    wl = pi.uniform_box((8, 8, 10), 1, 0.05, 0.1, 1, 7400, "cpu", tile=(4, 4, 4))
    boxes, Es, Bs, sl = _split(wl, (5, 5))        # interiors of 5 < 2 x 3 layers
    ctx = pic.pic_init(boxes, pic.PIC_FP64)
    f = pic.make_fields(boxes, Es, Bs, pic.PIC_FP64)
    with pytest.raises(pic.PicError) as e:
        pic.pic_slab_fill_guards(ctx, f, G)
    assert e.value.status == pic.PIC_ERR_ARG
    with pytest.raises(pic.PicError):
        pic.pic_slab_reduce_j(ctx, f, 2)
    pic.pic_free(ctx)
