"""pic_energy_noalloc (the entry point that allocates nothing) against
pic_energy through the C ABI: two calls in a row, the second on a smaller
input, each equal to pic_energy's result (same kernels and summation order:
bit-equal), and the species limit."""
import numpy as np
import pytest
import torch

import pic_inputs as pi
from pichelp import ensure_built
import paper_2303_12873_amd as pic

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    ensure_built()


def _setup(n, ppc, species, prec, seed):
    wl = pi.uniform_box(n, ppc, 0.05, 0.2, 2, seed, "cpu", tile=(4, 4, 4), fields="fourier",
                        species=species)
    ctx = pic.pic_init(wl.boxes, prec)
    f = pic.make_fields(wl.boxes, wl.E, wl.B, prec)
    sp = [pic.make_species(p, prec) for p in wl.species]
    return ctx, f, sp


@pytest.mark.parametrize("prec", (pic.PIC_FP64, pic.PIC_FP32_SPLIT))
def test_noalloc_energy_equals_pic_energy_twice(prec):
    big = _setup((24, 20, 16), 5, ("e", "i"), prec, 5100)
    small = _setup((6, 5, 4), 1, ("e",), prec, 5101)
    for ctx, f, sp in (big, small):
        ref = pic.pic_energy(ctx, f, sp, 0).cpu().numpy()
        out = torch.full((2 + len(sp),), float("nan"), dtype=torch.float64, device="cuda")
        pic.pic_energy_noalloc(ctx, f, sp, 0, out)
        got = out.cpu().numpy()
        assert np.all(np.isfinite(got))
        np.testing.assert_array_equal(got, ref)
        assert np.all(ref > 0)
    for ctx, _, _ in (big, small):
        pic.pic_free(ctx)


def test_noalloc_energy_rejects_too_many_species():
    ctx, f, sp = _setup((6, 5, 4), 1, ("e",), pic.PIC_FP64, 5102)
    out = torch.zeros(2 + 17, dtype=torch.float64, device="cuda")
    with pytest.raises(pic.PicError) as e:
        pic.pic_energy_noalloc(ctx, f, sp * 17, 0, out)
    assert e.value.status == pic.PIC_ERR_ARG
    pic.pic_free(ctx)
