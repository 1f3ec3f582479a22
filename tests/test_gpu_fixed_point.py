"""The split form's LDS current tile holds 64-bit fixed-point sums (a
per-tile power-of-two scale set by the largest charge factor of the tile's
particles).  Checked here: the sums of one tile do not depend on the order
of its particles (bit-identical J), weights spread over six decades stay
within the split tolerance of the oracle, and non-finite weights set the
range flag instead of reaching J."""
import numpy as np
import pytest
import torch

import oracle
import pic_inputs as pi
from pichelp import GpuRun, ensure_built, node_max_rel, rel_l2
import paper_2303_12873_amd as pic

pytestmark = pytest.mark.gpu

KERNELS = (pic.PIC_KERNEL_TILED, pic.PIC_KERNEL_BATCHED)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    ensure_built()


def _cluster(seed):
    """One 8^3 tile covering an 8^3 box; 4 particles in each of the cells
    3..4 along every axis, so every node they deposit to (1..7 per axis at
    order 3) is reached from one node of the LDS tile: the flush adds each
    global node once."""
    box = pi.Box(3, (8, 8, 8), pi.DT3, 3, (8, 8, 8))
    r = torch.arange(3, 5)
    cz, cy, cx = torch.meshgrid(r, r, r, indexing="ij")
    cells = (cx + 8 * (cy + 8 * cz)).reshape(-1)
    p = pi.particles_in_cells(box, cells, 4, 0.01, -1.0, 1.0, 0.2, seed, "cpu")
    g = torch.Generator().manual_seed(seed + 1)
    E = ((torch.rand((3, box.ncells), generator=g, dtype=torch.float64) - 0.5) * 0.02)
    B = ((torch.rand((3, box.ncells), generator=g, dtype=torch.float64) - 0.5) * 0.02)
    E = E.to(torch.float32).to(torch.float64)
    B = B.to(torch.float32).to(torch.float64)
    return pi.Workload("cluster_8cube_one_tile", [box], [p], [E], [B], steps=1)


def _box(seed, weights=None):
    wl = pi.uniform_box((12, 10, 9), 3, 0.05, 0.2, 3, seed, "cpu", tile=(4, 4, 4),
                        fields="fourier", species=("e", "i"))
    if weights is not None:
        for k, p in enumerate(wl.species):
            p.w = weights(p.np, k).to(torch.float32).to(torch.float64)
    return wl


def _permuted(wl, perm):
    p = wl.species[0]
    q = pi.Particles(p.q, p.m, p.x[:, perm].contiguous(), p.u[:, perm].contiguous(),
                     p.w[perm].contiguous(), p.cell[perm].contiguous(),
                     p.off[:, perm].contiguous(), p.box)
    return pi.Workload(wl.name, wl.boxes, [q], wl.E, wl.B, steps=1)


@pytest.mark.parametrize("kernel", KERNELS)
def test_tile_sums_do_not_depend_on_particle_order(kernel):
    wl = _cluster(7100)
    perm = torch.randperm(wl.species[0].np, generator=torch.Generator().manual_seed(3))
    wl2 = _permuted(wl, perm)
    Js = []
    assert wl.species[0].np == 32
    for w in (wl, wl2):
        run = GpuRun(w, pic.PIC_FP32_SPLIT, kernel=kernel, cell_order=-1)
        run.sort()
        pic.pic_advance(run.ctx, run.f, run.sp)
        run.check()
        Js.append(run.f.J.clone())
        run.free()
    assert torch.count_nonzero(Js[0]) > 0
    assert torch.equal(Js[0], Js[1])


@pytest.mark.parametrize("kernel", KERNELS)
def test_weights_over_six_decades_match_oracle(kernel):
    def weights(n, k):
        g = torch.Generator().manual_seed(11 + k)
        return 10.0 ** (-6.0 * torch.rand(n, generator=g, dtype=torch.float64)) * 0.01
    wl = _box(7200, weights=weights)
    box = wl.boxes[0]
    g = oracle.make_grid(box.dim, box.n, box.dx, box.dt, box.order)
    sps = [p.numpy() for p in wl.species]
    Jo = np.zeros_like(wl.E[0].numpy())
    oracle.particles_step(g, wl.E[0].numpy().copy(), wl.B[0].numpy().copy(), Jo, sps)
    run = GpuRun(wl, pic.PIC_FP32_SPLIT, kernel=kernel)
    run.sort()
    pic.pic_advance(run.ctx, run.f, run.sp)
    run.check()
    J = run.f.J.double().cpu().numpy()
    assert rel_l2(J, Jo) <= 1e-5 and node_max_rel(J, Jo) <= 1e-5, (rel_l2(J, Jo), node_max_rel(J, Jo))
    run.free()


@pytest.mark.parametrize("bad", (float("inf"), float("nan")))
@pytest.mark.parametrize("kernel", KERNELS)
def test_nonfinite_weight_sets_range_flag(kernel, bad):
    wl = _box(7300)
    wl.species[1].w[17] = bad
    run = GpuRun(wl, pic.PIC_FP32_SPLIT, kernel=kernel)
    run.sort()
    pic.pic_advance(run.ctx, run.f, run.sp)
    with pytest.raises(pic.PicError) as e:
        run.check()
    assert e.value.status == pic.PIC_ERR_RANGE
    run.check()          # flag cleared
    run.free()
