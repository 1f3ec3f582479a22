"""Laser-plasma boundaries on the GPU against the oracle: absorbing layers in
the Yee update, the laser antenna, and the moving window (circular z arrays
on the GPU, shifted arrays in the oracle) with particle removal and
injection, over whole steps of a small laser-plasma box."""
import math

import numpy as np
import pytest
import torch

import oracle
import pic_inputs as pi
from pichelp import ensure_built, node_max_rel, rel_l2
import paper_2303_12873_amd as pic

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    ensure_built()


@pytest.mark.parametrize("prec,tol", ((pic.PIC_FP64, 1e-12), (pic.PIC_FP32_SPLIT, 1e-6)))
@pytest.mark.parametrize("dim", (3, 2))
def test_absorbing_layers_parity(dim, prec, tol):
    n = (6, 5, 40) if dim == 3 else (6, 1, 40)
    box = pi.Box(dim, n, pi.DT3 if dim == 3 else pi.DT2, 1, (4, 4, 4) if dim == 3 else (4, 1, 4))
    E, B = pi.fourier_fields(box, 3, 0.1, 9100 + dim, "cpu")
    g = oracle.make_grid(dim, n, box.dx, box.dt, 1)
    a = oracle.absorber(8, 2.5, 3)
    Eo, Bo = E.numpy().copy(), B.numpy().copy()
    J = np.zeros_like(Eo)
    ctx = pic.pic_init([box], prec)
    pic.pic_set_absorber(ctx, 0, 8, 2.5, 3)
    f = pic.make_fields([box], [E], [B], prec)
    for _ in range(12):
        oracle.fdtd_step_absorb(g, Eo, Bo, J, a)
        pic.pic_fdtd_step(ctx, f)
    pic.pic_check(ctx)
    for t, ref in ((f.E, Eo), (f.B, Bo)):
        got = t.double().cpu().numpy()
        assert rel_l2(got, ref) <= tol and node_max_rel(got, ref) <= tol, (rel_l2(got, ref),)
    pic.pic_free(ctx)


def test_absorber_arguments_checked():
    box = pi.Box(3, (4, 4, 10), pi.DT3, 1, (4, 4, 4))
    ctx = pic.pic_init([box], pic.PIC_FP64)
    for args in ((6, 1.0, 3), (2, -1.0, 3), (2, 1.0, 9)):
        with pytest.raises(pic.PicError) as e:
            pic.pic_set_absorber(ctx, 0, *args)
        assert e.value.status == pic.PIC_ERR_ARG
    pic.pic_free(ctx)


def _inject(box, ppc, seed, frame_top, label0):
    """Seeded particles for one cell layer: positions in the window frame at
    layer frame_top, on the 2^-24 lattice, u_th = 0.02; weights are distinct
    labels starting at label0."""
    rng = np.random.default_rng(seed)
    nxy = box.n[0] * box.n[1]
    cells = np.repeat(np.arange(nxy), ppc)
    npart = cells.size
    off = rng.integers(0, 1 << 24, (3, npart)) * 2.0 ** -24
    x = np.stack([cells % box.n[0] + off[0],
                  (cells // box.n[0]) + off[1] if box.dim == 3 else np.zeros(npart),
                  frame_top + off[2]])
    u = np.float32(rng.normal(0.0, 0.02, (3, npart))).astype(np.float64)
    w = 2.0 ** -9 * (1.0 + (label0 + np.arange(npart)) * 2.0 ** -20)
    return pi.particles_from_positions(box, x, u, w, -1.0, 1.0)


@pytest.mark.parametrize("prec,kernel,tol", ((pic.PIC_FP64, pic.PIC_KERNEL_TILED, 1e-12),
                                             (pic.PIC_FP32_SPLIT, pic.PIC_KERNEL_BATCHED, 1e-5)))
def test_laser_plasma_box_with_antenna_absorber_and_moving_window(prec, kernel, tol):
    n = (8, 8, 48)
    box = pi.Box(3, n, pi.DT3, 2, (4, 4, 4))
    nz = n[2]
    # plasma in frame layers 4..40 (the window drops the lowest ones), laser
    # from an antenna at layer 12
    cells = torch.arange(box.ncells, dtype=torch.int64)
    cz = cells // (n[0] * n[1])
    plasma = cells[(cz >= 4) & (cz < 40)]
    e = pi.particles_in_cells(box, plasma, 2, 0.002, -1.0, 1.0, 0.02, 9200, "cpu")
    # distinct FP32-exact weights label the particles (matched by weight)
    e.w = 2.0 ** -9 * (1.0 + torch.arange(e.np, dtype=torch.float64) * 2.0 ** -20)
    E0, B0 = pi.zero_fields(box, "cpu")
    g = oracle.make_grid(3, n, box.dx, box.dt, 2)
    ab = oracle.absorber(8, 3.0, 3)
    an_args = dict(k=12, E0=0.05, omega=2 * math.pi / 20.0, waist=3.0, x0=4.0, y0=4.0,
                   t0=8.0, tau=5.0)
    an = oracle.antenna(**an_args)
    # oracle state (capacity for injections)
    cap = e.np + 400
    ref = e.numpy()
    xo = np.zeros((3, cap)); uo = np.zeros((3, cap)); wo = np.zeros(cap)
    xo[:, :e.np], uo[:, :e.np], wo[:e.np] = ref.x, ref.u, ref.w
    count = e.np
    Eo, Bo = E0.numpy().copy(), B0.numpy().copy()
    Jo = np.zeros_like(Eo)
    # GPU state
    ctx = pic.pic_init([box], prec, kernel=kernel)
    pic.pic_set_absorber(ctx, 0, 8, 3.0, 3)
    f = pic.make_fields([box], [E0], [B0], prec)
    sp = [pic.make_species(e, prec, capacity=cap)]

    class V:
        pass

    travelled, shifts = 0.0, 0
    for step in range(14):
        t = (step + 0.5) * box.dt
        # oracle
        v = V(); v.q, v.m = -1.0, 1.0
        v.x, v.u, v.w = np.ascontiguousarray(xo[:, :count]), np.ascontiguousarray(uo[:, :count]), \
            np.ascontiguousarray(wo[:count])
        oracle.particles_step(g, Eo, Bo, Jo, [v])
        xo[:, :count], uo[:, :count] = v.x, v.u
        oracle.antenna_add(g, Jo, an, t)
        oracle.fdtd_step_absorb(g, Eo, Bo, Jo, ab)
        # GPU
        pic.pic_sort_tiles(ctx, sp)
        pic.pic_advance(ctx, f, sp)
        pic.pic_antenna_add(ctx, f, 0, t=t, **an_args)
        pic.pic_fdtd_step(ctx, f)
        zoff_j = pic.pic_window_offset(ctx, 0)      # the frame of this step's J
        Jo_frame = Jo.copy()
        travelled += box.dt
        while travelled - shifts >= 1.0:
            new = _inject(box, 1, 9300 + shifts, nz - 1, e.np + shifts * 64)
            oracle.window_shift_fields(g, Eo, Bo)
            v = V(); v.q, v.m = -1.0, 1.0
            v.x, v.u, v.w = xo, uo, wo
            v.x = np.ascontiguousarray(xo[:, :count]); v.u = np.ascontiguousarray(uo[:, :count])
            v.w = np.ascontiguousarray(wo[:count])
            m = oracle.window_shift_particles(g, v)
            xo[:, :m], uo[:, :m], wo[:m] = v.x[:, :m], v.u[:, :m], v.w[:m]
            xo[:, m:m + new.np] = new.x.numpy()
            uo[:, m:m + new.np] = new.u.numpy()
            wo[m:m + new.np] = new.w.numpy()
            count = m + new.np
            inj = pic.make_species(new, prec)
            pic.pic_window_shift(ctx, f, sp, 0, [inj])
            shifts += 1
        pic.pic_check(ctx)
    assert shifts >= 7
    zoff = pic.pic_window_offset(ctx, 0)
    assert zoff == shifts % nz

    def frame(t, zo):
        a = t.double().cpu().numpy().reshape(3, nz, n[1], n[0])
        return np.roll(a, -zo, axis=1).reshape(3, -1)

    # E, B in the current frame; J (not moved by a shift) in the frame of
    # the step that deposited it
    for t, zo, ref_f, name in ((f.E, zoff, Eo, "E"), (f.B, zoff, Bo, "B"),
                               (f.J, zoff_j, Jo_frame, "J")):
        got = frame(t, zo)
        assert rel_l2(got, ref_f) <= tol, (name, rel_l2(got, ref_f))
        assert node_max_rel(got, ref_f) <= tol, (name, node_max_rel(got, ref_f))
    assert np.max(np.abs(Eo[0])) > 1e-3          # the laser is in the box
    s = sp[0]
    assert s.np == count
    if s.x is not None:
        xg = s.x[:, :s.np].double().cpu().numpy().copy()
    else:
        cell = s.cell[:s.np].long().cpu().numpy()
        off = s.off[:, :s.np].double().cpu().numpy()
        xg = np.stack([cell % n[0] + off[0], (cell // n[0]) % n[1] + off[1],
                       cell // (n[0] * n[1]) + off[2]])
    xg[2] = np.mod(xg[2] - zoff, nz)
    ug = s.u[:, :s.np].double().cpu().numpy()
    wg = s.w[:s.np].double().cpu().numpy()
    og, oo = np.argsort(wg, kind="stable"), np.argsort(wo[:count], kind="stable")
    np.testing.assert_array_equal(wg[og], wo[:count][oo])      # every particle once
    d = xg[:, og] - xo[:, :count][:, oo]
    d -= np.array(n, dtype=np.float64)[:, None] * np.round(d / np.array(n, dtype=np.float64)[:, None])
    assert np.max(np.abs(d)) <= (1e-12 if prec == pic.PIC_FP64 else 1e-5) * nz
    assert rel_l2(ug[:, og], uo[:, :count][:, oo]) <= tol
    pic.pic_free(ctx)
