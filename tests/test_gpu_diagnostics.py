"""The library's FP64 energy reductions against the oracle's energies, and
the step-graph cache when a context's scratch buffers are reallocated."""
import numpy as np
import pytest
import torch

import oracle
import pic_inputs as pi
from pichelp import GpuRun, ensure_built, periodic_diff, rel_l2
import paper_2303_12873_amd as pic

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    ensure_built()


@pytest.mark.parametrize("prec", (pic.PIC_FP64, pic.PIC_FP32_SPLIT))
@pytest.mark.parametrize("dim", (3, 2))
def test_energy_matches_oracle(prec, dim):
    # inputs are FP32-representable, so both forms hold the same values and
    # only the order of the FP64 sums differs
    wl = pi.uniform_box((12, 10, 9), 3, 0.05, 0.3, 2, 4100 + dim, "cpu", tile=(4, 4, 4),
                        fields="fourier", dim=dim, species=("e", "i"))
    box = wl.boxes[0]
    g = oracle.make_grid(box.dim, box.n, box.dx, box.dt, box.order)
    E = wl.E[0].numpy().copy()
    B = wl.B[0].numpy().copy()
    run = GpuRun(wl, prec)
    out = pic.pic_energy(run.ctx, run.f, run.sp, 0).cpu().numpy()
    eo = oracle.field_energy(g, E, np.zeros_like(B))
    bo = oracle.field_energy(g, np.zeros_like(E), B)
    ko = [oracle.kinetic_energy(p.numpy()) for p in wl.species]
    assert abs(out[0] - eo) <= 1e-13 * eo, (out[0], eo)
    assert abs(out[1] - bo) <= 1e-13 * bo, (out[1], bo)
    for s in range(2):
        assert abs(out[2 + s] - ko[s]) <= 1e-13 * ko[s], (s, out[2 + s], ko[s])
    run.free()


def test_energy_species_of_other_box_is_zero():
    wl = pi.c4("cpu", nboxes=2, l_range=(12, 16), big=(16, 16, 16))
    boxes = wl.boxes
    ctx = pic.pic_init(boxes, pic.PIC_FP64)
    f = pic.make_fields(boxes, wl.E, wl.B, pic.PIC_FP64)
    sp = [pic.make_species(p, pic.PIC_FP64) for p in wl.species]
    out = pic.pic_energy(ctx, f, sp, 1).cpu().numpy()
    for s, p in enumerate(wl.species):
        if p.box != 1:
            assert out[2 + s] == 0.0
        else:
            ko = oracle.kinetic_energy(p.numpy())
            assert abs(out[2 + s] - ko) <= 1e-13 * ko
    pic.pic_free(ctx)


@pytest.mark.parametrize("prec", (pic.PIC_FP64, pic.PIC_FP32_SPLIT))
def test_graph_cache_survives_scratch_growth(prec):
    """Species set A, then {A, a larger B} (the sort and per-species scratch
    grow and are reallocated), then A again on one context: every pic_step
    replay must equal the same work issued eagerly on a second context."""
    wl = pi.uniform_box((12, 12, 12), 2, 0.05, 0.1, 2, 4300, "cpu", tile=(4, 4, 4),
                        fields="fourier", species=("e",))
    big = pi.uniform_box((12, 12, 12), 9, 0.05, 0.1, 2, 4301, "cpu", tile=(4, 4, 4),
                         species=("i",))
    box = wl.boxes[0]
    pa, pb = wl.species[0], big.species[0]
    tol = 1e-12 if prec == pic.PIC_FP64 else 1e-5

    def setup():
        ctx = pic.pic_init([box], prec)
        f = pic.make_fields([box], wl.E, wl.B, prec)
        return ctx, f, pic.make_species(pa, prec), pic.make_species(pb, prec)

    cg, fg, ag, bg = setup()
    ce, fe, ae, be = setup()
    seq = [[0], [0], [0, 1], [0, 1], [0], [0]]
    for k, sel in enumerate(seq):
        sg = [(ag, bg)[i] for i in sel]
        se = [(ae, be)[i] for i in sel]
        sort = k == 0 or sel != seq[k - 1]
        pic.pic_step(cg, fg, sg, sort=sort)
        if sort:
            pic.pic_sort_tiles(ce, se)
        pic.pic_advance(ce, fe, se)
        pic.pic_fdtd_step(ce, fe)
        pic.pic_check(cg)
        pic.pic_check(ce)
        for a, b in ((fg.E, fe.E), (fg.B, fe.B), (fg.J, fe.J)):
            assert rel_l2(a.double().cpu().numpy(), b.double().cpu().numpy()) <= tol, k
        for x, y in zip(sg, se):
            ux, uy = x.u.double().cpu().numpy(), y.u.double().cpu().numpy()
            assert rel_l2(ux, uy) <= tol, k
    for c in (cg, ce):
        pic.pic_free(c)


@pytest.mark.parametrize("prec", (pic.PIC_FP64, pic.PIC_FP32_SPLIT))
def test_slice_moments_match_oracle(prec):
    wl = pi.uniform_box((7, 6, 11), 4, 0.05, 0.3, 2, 4500, "cpu", tile=(4, 4, 4),
                        species=("e", "i"))
    box = wl.boxes[0]
    g = oracle.make_grid(box.dim, box.n, box.dx, box.dt, box.order)
    run = GpuRun(wl, prec)
    out = pic.pic_slice_moments(run.ctx, run.sp, 0, box.n[2]).cpu().numpy()
    run.check()
    for s, p in enumerate(wl.species):
        ref = oracle.slice_moments(g, p.numpy())
        np.testing.assert_allclose(out[s], ref, rtol=1e-12, atol=1e-18)
    run.free()
