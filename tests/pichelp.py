"""Shared helpers of the test-suite: build-if-missing, running the GPU path
through the C ABI binding, and the error measures used by the parity bars.

The HIP path and the oracle never share arithmetic: this module only moves
arrays between them and compares results.
"""
from __future__ import annotations

import os
import sys

import numpy as np
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import paper_2303_12873_amd as pic  # noqa: E402


def ensure_built():
    if not os.path.exists(pic.LIB_PATH):
        from paper_2303_12873_amd.build import build
        build()


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b.ravel())
    return float(np.linalg.norm((a - b).ravel()) / (nb if nb > 0 else 1.0))


def node_max_rel(a, b):
    """max over nodes |a - b| / max |b| (node-wise bound beside rel_l2)."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    mb = np.max(np.abs(b)) if b.size else 0.0
    return float(np.max(np.abs(a - b)) / (mb if mb > 0 else 1.0)) if b.size else 0.0


def periodic_diff(a, b, L):
    """a - b folded into [-L/2, L/2) per row (positions in cell units)."""
    d = np.asarray(a) - np.asarray(b)
    L = np.asarray(L, dtype=np.float64).reshape(-1, *([1] * (d.ndim - 1)))
    return d - L * np.round(d / L)


class GpuRun:
    """One box (or several) and its species on the GPU, FP64 or split form."""

    def __init__(self, wl, precision, kernel=None, block=0, chunk=0, wg_per_cu=0, stream=None,
                 lane_stride=0, cell_order=0, quad_spread=0, pad=0, margin=0):
        ensure_built()
        self.wl = wl
        self.prec = precision
        self.ctx = pic.pic_init(wl.boxes, precision, stream=stream, kernel=kernel, block=block,
                                chunk=chunk, wg_per_cu=wg_per_cu, lane_stride=lane_stride,
                                cell_order=cell_order, quad_spread=quad_spread, pad=pad,
                                margin=margin)
        self.f = pic.make_fields(wl.boxes, wl.E, wl.B, precision)
        self.sp = [pic.make_species(p, precision) for p in wl.species]
        self.kernel = kernel if kernel is not None else (
            pic.PIC_KERNEL_TILED if precision == pic.PIC_FP64 else pic.PIC_KERNEL_BATCHED)

    def sort(self):
        """Sort and keep track of each particle's original index."""
        perms = [torch.empty(sp.np, dtype=torch.int32, device="cuda") for sp in self.sp]
        pic.pic_sort_tiles(self.ctx, self.sp, perm_out=perms)
        if not hasattr(self, "ident"):
            self.ident = [torch.arange(sp.np, device="cuda") for sp in self.sp]
        self.ident = [idn[pm.long()] for idn, pm in zip(self.ident, perms)]

    def particles(self, split=False):
        if split:
            pic.pic_gather_push(self.ctx, self.f, self.sp)
            pic.pic_deposit_J(self.ctx, self.f, self.sp)
        else:
            pic.pic_advance(self.ctx, self.f, self.sp)

    def step(self, sort=False, split=False):
        if sort or (self.kernel != pic.PIC_KERNEL_DIRECT and not getattr(self, "_sorted", False)):
            self.sort()
            self._sorted = True
        self.particles(split)
        pic.pic_fdtd_step(self.ctx, self.f)

    def check(self):
        pic.pic_check(self.ctx)

    def energy(self, b=0):
        """(field energy, kinetic energy of all species of box b) from the
        library's FP64 device reductions."""
        out = pic.pic_energy(self.ctx, self.f, self.sp, b).cpu().numpy()
        return float(out[0] + out[1]), float(np.sum(out[2:]))

    def rho_np(self, b=0):
        box = self.wl.boxes[b]
        r = torch.zeros(box.ncells, dtype=torch.float64, device="cuda")
        pic.pic_deposit_rho(self.ctx, self.sp, b, r)
        return r.cpu().numpy()

    def fields_np(self, b=0):
        box = self.wl.boxes[b]
        get = lambda t: self.f.box_view(t, b, box.ncells).double().cpu().numpy()
        return get("E"), get("B"), get("J")

    def original_order(self, s=0):
        """Index array that puts GPU particle arrays back in input order."""
        if not hasattr(self, "ident"):
            return np.arange(self.sp[s].np)
        return np.argsort(self.ident[s].cpu().numpy(), kind="stable")

    def state_np(self, s=0):
        """(x, u) in the original particle order, FP64 numpy."""
        o = self.original_order(s)
        return self.positions_np(s)[:, o], self.sp[s].u.double().cpu().numpy()[:, o]

    def positions_np(self, s=0):
        """Positions (3, np) FP64 in cell units, in the current GPU order."""
        sp = self.sp[s]
        if sp.x is not None:
            return sp.x.cpu().numpy()
        box = self.wl.boxes[sp.box]
        cell = sp.cell.long().cpu().numpy()
        cx = cell % box.n[0]
        cy = (cell // box.n[0]) % box.n[1]
        cz = cell // (box.n[0] * box.n[1])
        off = sp.off.double().cpu().numpy()
        return np.stack([cx + off[0], cy + off[1], cz + off[2]])

    def free(self):
        pic.pic_free(self.ctx)
