"""Host-side checks of the C ABI that need no GPU: the library builds and
exports every entry point declared in include/libpic.h, and argument
validation in pic_init rejects bad boxes before any device call."""
import ctypes as C
import os
import re

import pytest

from pichelp import ROOT, ensure_built
import paper_2303_12873_amd as pic


def _declared():
    src = open(os.path.join(ROOT, "include", "libpic.h")).read()
    return sorted(set(re.findall(r"\b(pic_[a-z_A-Z]+)\s*\(", src)))


def test_header_declares_the_five_hot_path_calls():
    names = _declared()
    for n in ("pic_init", "pic_sort_tiles", "pic_gather_push", "pic_deposit_J", "pic_fdtd_step"):
        assert n in names


def test_library_exports_every_declared_symbol():
    ensure_built()
    L = C.CDLL(pic.LIB_PATH)
    for n in _declared():
        assert hasattr(L, n), n
    assert set(_declared()) <= set(pic.EXPORTED)


class _Box:
    def __init__(self, **kw):
        self.dim, self.n, self.dx, self.dt, self.order, self.tile = 3, (8, 8, 8), (1, 1, 1), 0.5, 1, (4, 4, 4)
        self.__dict__.update(kw)

    @property
    def ncells(self):
        return self.n[0] * self.n[1] * self.n[2]


@pytest.mark.parametrize("kw,status", [
    (dict(order=4), pic.PIC_ERR_ARG),
    (dict(order=0), pic.PIC_ERR_ARG),
    (dict(dim=1), pic.PIC_ERR_ARG),
    (dict(dt=0.58), pic.PIC_ERR_CFL),            # 0.99/sqrt(3) < 0.58
    (dict(dt=-1.0), pic.PIC_ERR_ARG),
    (dict(n=(8, 0, 8)), pic.PIC_ERR_ARG),
    (dict(tile=(4, 17, 4)), pic.PIC_ERR_ARG),
    (dict(dim=2, n=(8, 2, 8), dt=0.5), pic.PIC_ERR_ARG),
    (dict(dim=2, n=(8, 1, 8), tile=(4, 1, 4), dt=0.71), pic.PIC_ERR_CFL),
    (dict(dx=(1, 0, 1)), pic.PIC_ERR_ARG),
])
def test_pic_init_rejects_bad_boxes_on_the_host(kw, status):
    ensure_built()
    with pytest.raises(pic.PicError) as e:
        pic.pic_init([_Box(**kw)], pic.PIC_FP64, stream=0)
    assert e.value.status == status


@pytest.mark.parametrize("kw", [dict(block=96), dict(block=2048), dict(lane_stride=65),
                                dict(cell_order=5), dict(cell_order=-2), dict(pad=3),
                                dict(pad=-2), dict(quad_spread=2), dict(wg_per_cu=65),
                                dict(margin=1), dict(margin=-2),
                                dict(kernel=3)])
def test_pic_init_rejects_bad_tuning_on_the_host(kw):
    ensure_built()
    args = dict(kernel=pic.PIC_KERNEL_BATCHED)
    args.update(kw)
    with pytest.raises(pic.PicError) as e:
        pic.pic_init([_Box()], pic.PIC_FP32_SPLIT, stream=0, **args)
    assert e.value.status == pic.PIC_ERR_ARG


def test_mixed_orders_rejected():
    ensure_built()
    with pytest.raises(pic.PicError) as e:
        pic.pic_init([_Box(), _Box(order=2)], pic.PIC_FP64, stream=0)
    assert e.value.status == pic.PIC_ERR_ARG


def test_status_strings():
    ensure_built()
    for s in range(7):
        assert pic.pic_status_str(s)
