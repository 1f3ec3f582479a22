"""MI355X-native hot path of an explicit electromagnetic PIC step.

Thin ctypes binding of ``libpic.so`` (C ABI in ``include/libpic.h``): the
functions below carry the same names as the C entry points and only marshal
arguments (torch tensors -> device pointers, Python lists -> C structs).
Every step of the path runs in the library's HIP kernels.  PyTorch supplies
device memory and the stream.

If ``libpic.so`` is missing the import of this module still works, but the
first call raises: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import List, Optional, Sequence

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpic.so")

PIC_OK, PIC_ERR_ARG, PIC_ERR_CFL, PIC_ERR_OOM, PIC_ERR_DEVICE, PIC_ERR_RANGE, PIC_ERR_STATE = range(7)
PIC_FP64, PIC_FP32_SPLIT = 0, 1
PIC_KERNEL_DIRECT, PIC_KERNEL_TILED, PIC_KERNEL_BATCHED = 0, 1, 2

EXPORTED = ["pic_init", "pic_sort_tiles", "pic_gather_push", "pic_deposit_J", "pic_advance",
            "pic_fdtd_step", "pic_step", "pic_deposit_rho", "pic_div_edge", "pic_energy", "pic_check",
            "pic_free", "pic_status_str", "pic_last_error", "pic_device_cus", "pic_set_timing",
            "pic_kernel_ms"]


class pic_box_desc(C.Structure):
    _fields_ = [("dim", C.c_int32), ("n", C.c_int32 * 3), ("dx", C.c_double * 3),
                ("dt", C.c_double), ("order", C.c_int32), ("tile", C.c_int32 * 3),
                ("cell_base", C.c_int64)]


class pic_tuning(C.Structure):
    _fields_ = [("kernel", C.c_int32), ("block", C.c_int32), ("chunk", C.c_int32),
                ("wg_per_cu", C.c_int32), ("lane_stride", C.c_int32), ("pad", C.c_int32),
                ("cell_order", C.c_int32), ("quad_spread", C.c_int32), ("margin", C.c_int32)]


class pic_fields(C.Structure):
    _fields_ = [("E", C.c_void_p * 3), ("B", C.c_void_p * 3), ("J", C.c_void_p * 3)]


class pic_species(C.Structure):
    _fields_ = [("np", C.c_int64), ("q", C.c_double), ("m", C.c_double), ("box", C.c_int32),
                ("x", C.c_void_p * 3), ("cell", C.c_void_p), ("off", C.c_void_p * 3),
                ("u", C.c_void_p * 3), ("w", C.c_void_p)]


class PicError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{msg} (status {status})")
        self.status = status


_lib = None


def lib():
    """Load libpic.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built: run `python -m paper_2303_12873_amd.build`")
        L = C.CDLL(LIB_PATH)
        P, I = C.c_void_p, C.c_int32
        L.pic_init.argtypes = [C.POINTER(P), C.POINTER(pic_box_desc), I, I, P, C.POINTER(pic_tuning)]
        L.pic_sort_tiles.argtypes = [P, C.POINTER(pic_species), I, P, P, P]
        for n in ("pic_gather_push", "pic_deposit_J", "pic_advance"):
            getattr(L, n).argtypes = [P, C.POINTER(pic_fields), C.POINTER(pic_species), I]
        L.pic_fdtd_step.argtypes = [P, C.POINTER(pic_fields)]
        L.pic_step.argtypes = [P, C.POINTER(pic_fields), C.POINTER(pic_species), I, I]
        L.pic_deposit_rho.argtypes = [P, C.POINTER(pic_species), I, I, P]
        L.pic_div_edge.argtypes = [P, I, P, P]
        L.pic_energy.argtypes = [P, C.POINTER(pic_fields), C.POINTER(pic_species), I, I, P]
        L.pic_check.argtypes = [P]
        L.pic_free.argtypes = [P]
        L.pic_status_str.argtypes = [I]
        L.pic_status_str.restype = C.c_char_p
        L.pic_last_error.restype = C.c_char_p
        L.pic_device_cus.argtypes = [P]
        L.pic_set_timing.argtypes = [P, I]
        L.pic_kernel_ms.argtypes = [P, C.POINTER(C.c_float)]
        for n in EXPORTED:
            if n not in ("pic_status_str", "pic_last_error", "pic_device_cus"):
                getattr(L, n).restype = C.c_int
        _lib = L
    return _lib


def _check(st):
    if st != PIC_OK:
        msg = lib().pic_last_error().decode()
        raise PicError(st, msg or lib().pic_status_str(st).decode())


def _ptr(t: Optional[torch.Tensor]):
    if t is None:
        return None
    if not t.is_contiguous():
        raise ValueError("tensors passed to libpic must be contiguous")
    return t.data_ptr()


# ------------------------------------------------------------------ containers

@dataclass
class DeviceFields:
    """E, B (FP64 or FP32) and J (FP64), shape (3, total cells); box b at
    ``cell_base[b]``."""
    E: torch.Tensor
    B: torch.Tensor
    J: torch.Tensor
    cell_base: List[int]

    def c(self) -> pic_fields:
        f = pic_fields()
        for d in range(3):
            f.E[d] = _ptr(self.E[d])
            f.B[d] = _ptr(self.B[d])
            f.J[d] = _ptr(self.J[d])
        return f

    def box_view(self, comp: str, b: int, ncells: int) -> torch.Tensor:
        t = getattr(self, comp)
        return t[:, self.cell_base[b]:self.cell_base[b] + ncells]


def make_fields(boxes, E_list, B_list, precision: int, device="cuda") -> DeviceFields:
    """Concatenate per-box initial fields (FP64 tensors) on the device."""
    ft = torch.float64 if precision == PIC_FP64 else torch.float32
    bases, tot = [], 0
    for b in boxes:
        bases.append(tot)
        tot += b.ncells
    E = torch.empty((3, tot), dtype=ft, device=device)
    B = torch.empty((3, tot), dtype=ft, device=device)
    J = torch.zeros((3, tot), dtype=torch.float64, device=device)
    for b, base, e, bb in zip(boxes, bases, E_list, B_list):
        E[:, base:base + b.ncells].copy_(e)
        B[:, base:base + b.ncells].copy_(bb)
    return DeviceFields(E, B, J, bases)


@dataclass
class DeviceSpecies:
    """One species' particle arrays on the device, FP64 or split form."""
    q: float
    m: float
    box: int
    precision: int
    u: torch.Tensor
    w: torch.Tensor
    x: Optional[torch.Tensor] = None       # FP64: (3, np)
    cell: Optional[torch.Tensor] = None    # split: (np,) int32
    off: Optional[torch.Tensor] = None     # split: (3, np) float32

    @property
    def np(self) -> int:
        return int(self.w.shape[0])

    def c(self) -> pic_species:
        s = pic_species()
        s.np = self.np
        s.q = self.q
        s.m = self.m
        s.box = self.box
        for d in range(3):
            s.u[d] = _ptr(self.u[d])
            if self.x is not None:
                s.x[d] = _ptr(self.x[d])
            if self.off is not None:
                s.off[d] = _ptr(self.off[d])
        s.cell = _ptr(self.cell)
        s.w = _ptr(self.w)
        return s


def make_species(p, precision: int, box: int = None, device="cuda") -> DeviceSpecies:
    """Device copy of a ``pic_inputs.Particles`` in the requested form (always
    new storage: the kernels update it in place)."""
    b = p.box if box is None else box

    def cp(t, dt):
        return t.to(device=device, dtype=dt, copy=True).contiguous()

    if precision == PIC_FP64:
        return DeviceSpecies(p.q, p.m, b, precision, cp(p.u, torch.float64), cp(p.w, torch.float64),
                             x=cp(p.x, torch.float64))
    return DeviceSpecies(p.q, p.m, b, precision, cp(p.u, torch.float32), cp(p.w, torch.float32),
                         cell=cp(p.cell, torch.int32), off=cp(p.off, torch.float32))


def _species_array(species: Sequence[DeviceSpecies]):
    arr = (pic_species * max(1, len(species)))(*[s.c() for s in species])
    return arr


def _ptr_array(ts):
    if ts is None:
        return None
    arr = (C.c_void_p * len(ts))(*[_ptr(t) if t is not None else None for t in ts])
    return C.cast(arr, C.c_void_p), arr


# ------------------------------------------------------------------ C ABI names

def pic_init(boxes, precision: int, stream=None, kernel: Optional[int] = None, block: int = 0,
             chunk: int = 0, wg_per_cu: int = 0, lane_stride: int = 0, pad: int = 0,
             cell_order: int = 0, quad_spread: int = 0, margin: int = 0):
    """boxes: objects with dim, n, dx, dt, order, tile (``pic_inputs.Box``).
    Returns an opaque context handle (int)."""
    descs = (pic_box_desc * len(boxes))()
    base = 0
    for i, b in enumerate(boxes):
        d = descs[i]
        d.dim = b.dim
        for k in range(3):
            d.n[k] = b.n[k]
            d.dx[k] = b.dx[k]
            d.tile[k] = b.tile[k]
        d.dt = b.dt
        d.order = b.order
        d.cell_base = base
        base += b.ncells
    tun = None
    if (kernel is not None or block or chunk or wg_per_cu or lane_stride or pad or cell_order
            or quad_spread or margin):
        tun = pic_tuning()
        tun.kernel = (PIC_KERNEL_TILED if precision == PIC_FP64 else PIC_KERNEL_BATCHED) \
            if kernel is None else kernel
        tun.block, tun.chunk, tun.wg_per_cu = block, chunk, wg_per_cu
        tun.lane_stride = lane_stride
        tun.pad = pad
        tun.cell_order = cell_order
        tun.quad_spread = quad_spread
        tun.margin = margin
    if stream is None:
        stream = torch.cuda.current_stream().cuda_stream
    h = C.c_void_p()
    _check(lib().pic_init(C.byref(h), descs, len(boxes), precision, C.c_void_p(stream),
                          C.byref(tun) if tun is not None else None))
    return h.value


def pic_sort_tiles(ctx, species, perm_out=None, key_out=None, tile_offset_out=None):
    arr = _species_array(species)
    po = _ptr_array(perm_out)
    ko = _ptr_array(key_out)
    oo = _ptr_array(tile_offset_out)
    _check(lib().pic_sort_tiles(ctx, arr, len(species), po[0] if po else None,
                                ko[0] if ko else None, oo[0] if oo else None))


def pic_gather_push(ctx, fields: DeviceFields, species):
    f = fields.c()
    _check(lib().pic_gather_push(ctx, C.byref(f), _species_array(species), len(species)))


def pic_deposit_J(ctx, fields: DeviceFields, species):
    f = fields.c()
    _check(lib().pic_deposit_J(ctx, C.byref(f), _species_array(species), len(species)))


def pic_advance(ctx, fields: DeviceFields, species):
    f = fields.c()
    _check(lib().pic_advance(ctx, C.byref(f), _species_array(species), len(species)))


def pic_fdtd_step(ctx, fields: DeviceFields):
    f = fields.c()
    _check(lib().pic_fdtd_step(ctx, C.byref(f)))


def pic_step(ctx, fields: DeviceFields, species, sort: bool):
    f = fields.c()
    _check(lib().pic_step(ctx, C.byref(f), _species_array(species), len(species), int(bool(sort))))


def pic_deposit_rho(ctx, species, box: int, rho: torch.Tensor):
    _check(lib().pic_deposit_rho(ctx, _species_array(species), len(species), box, _ptr(rho)))


def pic_div_edge(ctx, box: int, v: Sequence[torch.Tensor], out: torch.Tensor):
    arr = (C.c_void_p * 3)(*[_ptr(t) for t in v])
    _check(lib().pic_div_edge(ctx, box, C.cast(arr, C.c_void_p), _ptr(out)))


def pic_energy(ctx, fields: DeviceFields, species, box: int = 0, out: torch.Tensor = None):
    """FP64 energies of one box on the device: returns ``out`` (2 + nsp
    doubles): 1/2 sum E.E dV, 1/2 sum B.B dV, then sum w m (gamma - 1) per
    species (0 for species of other boxes)."""
    if out is None:
        out = torch.empty(2 + len(species), dtype=torch.float64, device=fields.E.device)
    f = fields.c()
    _check(lib().pic_energy(ctx, C.byref(f), _species_array(species), len(species), box,
                            _ptr(out)))
    return out


def pic_check(ctx):
    _check(lib().pic_check(ctx))


def pic_free(ctx):
    _check(lib().pic_free(ctx))


def pic_device_cus(ctx) -> int:
    return int(lib().pic_device_cus(ctx))


def pic_set_timing(ctx, on: bool = True):
    _check(lib().pic_set_timing(ctx, int(bool(on))))


def pic_kernel_ms(ctx) -> float:
    ms = C.c_float()
    _check(lib().pic_kernel_ms(ctx, C.byref(ms)))
    return float(ms.value)


def pic_status_str(status: int) -> str:
    return lib().pic_status_str(status).decode()
