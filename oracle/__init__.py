"""Plain FP64 CPU oracle of the explicit electromagnetic PIC step.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import this package.  The
product library never loads it; it shares no code with the GPU path.

The arithmetic lives in ``pic_oracle.c`` (plain C, FP64, loops in particle
index order); this module compiles it with gcc and marshals numpy arrays
through ctypes.  Each C function cites the published method it follows:
B-spline shapes, Boris (1970), Esirkepov (2001), Yee (1966) -- the four steps
of the fully-kinetic explicit EM PIC method the paper names in Sec. II and
Sec. IV.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pic_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build() -> str:
    """Compile the oracle (always recompiles)."""
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off",
           "-fno-fast-math", "-o", _LIB + ".tmp", _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class Grid(C.Structure):
    _fields_ = [("dim", C.c_int32), ("n", C.c_int32 * 3), ("dx", C.c_double * 3),
                ("dt", C.c_double), ("order", C.c_int32)]


class Species(C.Structure):
    _fields_ = [("np", C.c_int64), ("q", C.c_double), ("m", C.c_double),
                ("x", C.c_void_p * 3), ("u", C.c_void_p * 3), ("w", C.c_void_p)]


class Absorber(C.Structure):
    _fields_ = [("cells", C.c_int32), ("sigma_max", C.c_double), ("power", C.c_int32)]


class Antenna(C.Structure):
    _fields_ = [("k", C.c_int32), ("E0", C.c_double), ("omega", C.c_double),
                ("waist", C.c_double), ("x0", C.c_double), ("y0", C.c_double),
                ("t0", C.c_double), ("tau", C.c_double)]


_P = C.c_void_p
_D = C.c_double
_I = C.c_int32


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = C.CDLL(_LIB)
        L.orc_shape.argtypes = [_I, _D]
        L.orc_shape.restype = _D
        L.orc_gather.argtypes = [C.POINTER(Grid), _P, _P, _P, _P, _P]
        L.orc_boris.argtypes = [_D, _D, _D, _P, _P, _P]
        L.orc_deposit.argtypes = [C.POINTER(Grid), _P, _D, _D, _P, _P, _D]
        L.orc_faraday.argtypes = [C.POINTER(Grid), _P, _P, _D]
        L.orc_ampere.argtypes = [C.POINTER(Grid), _P, _P, _P, _D]
        L.orc_fdtd_step.argtypes = [C.POINTER(Grid), _P, _P, _P]
        L.orc_wrap.argtypes = [_D, _D]
        L.orc_wrap.restype = _D
        L.orc_particles_step.argtypes = [C.POINTER(Grid), _P, _P, _P, C.POINTER(Species), _I]
        L.orc_pic_step.argtypes = [C.POINTER(Grid), _P, _P, _P, C.POINTER(Species), _I]
        L.orc_rho.argtypes = [C.POINTER(Grid), _P, C.POINTER(Species)]
        L.orc_div_j.argtypes = [C.POINTER(Grid), _P, _P]
        L.orc_field_energy.argtypes = [C.POINTER(Grid), _P, _P]
        L.orc_field_energy.restype = _D
        L.orc_kinetic_energy.argtypes = [C.POINTER(Species)]
        L.orc_kinetic_energy.restype = _D
        L.orc_tile_keys.argtypes = [C.POINTER(Grid), _P, C.POINTER(Species), _P]
        L.orc_stable_sort.argtypes = [C.c_int64, _P, _I, _P, _P, _P]
        L.orc_cell_order_keys.argtypes = [C.POINTER(Grid), _P, _I, C.POINTER(Species), _P]
        L.orc_stable_perm.argtypes = [C.c_int64, _P, _P]
        L.orc_quad_order.argtypes = [C.c_int64, _P, _I, _P]
        L.orc_tile_cell_keys.argtypes = [C.POINTER(Grid), _P, _I, C.POINTER(Species), _P]
        L.orc_absorber_sigma.argtypes = [C.POINTER(Absorber), _D, _D]
        L.orc_absorber_sigma.restype = _D
        L.orc_fdtd_step_absorb.argtypes = [C.POINTER(Grid), _P, _P, _P, C.POINTER(Absorber), _D]
        L.orc_antenna_add.argtypes = [C.POINTER(Grid), _P, C.POINTER(Antenna), _D]
        L.orc_window_shift_fields.argtypes = [C.POINTER(Grid), _P, _P]
        L.orc_window_shift_particles.argtypes = [C.POINTER(Grid), C.POINTER(Species)]
        L.orc_window_shift_particles.restype = C.c_int64
        L.orc_es_field.argtypes = [C.POINTER(Grid), _P, _P]
        L.orc_vay.argtypes = [_D, _D, _D, _P, _P, _P]
        L.orc_slice_moments.argtypes = [C.POINTER(Grid), C.POINTER(Species), _I, _P]
        L.orc_rank_major.argtypes = [C.c_int64, _P, _I, _I, _P]
        L.orc_gather_galerkin.argtypes = [C.POINTER(Grid), _P, _P, _P, _P, _P]
        L.orc_particles_step_opts.argtypes = [C.POINTER(Grid), _P, _P, _P, C.POINTER(Species), _I,
                                              _I, _I]
        L.orc_es_particles_step.argtypes = [C.POINTER(Grid), _P, C.POINTER(Species), _I]
        _lib = L
    return _lib


# ------------------------------------------------------------------ marshalling

def _f64(a):
    a = np.asarray(a)
    if a.dtype != np.float64 or not a.flags.c_contiguous:
        raise TypeError("oracle arrays must be C-contiguous float64")
    return a


def make_grid(dim, n, dx, dt, order) -> Grid:
    g = Grid()
    g.dim = int(dim)
    for d in range(3):
        g.n[d] = int(n[d])
        g.dx[d] = float(dx[d])
    g.dt = float(dt)
    g.order = int(order)
    return g


class _FieldPtrs:
    """Keeps three component arrays alive and exposes a ``double*[3]``."""

    def __init__(self, comps):
        self.comps = [_f64(c) for c in comps]
        self.arr = (C.c_void_p * 3)(*[c.ctypes.data for c in self.comps])

    @property
    def ptr(self):
        return C.cast(self.arr, C.c_void_p)


def _species_struct(sp):
    """``sp`` is any object with q, m, x (3,np), u (3,np), w (np) float64."""
    s = Species()
    x = sp.x
    s.np = int(x.shape[1])
    s.q = float(sp.q)
    s.m = float(sp.m)
    for d in range(3):
        s.x[d] = _f64(x[d]).ctypes.data
        s.u[d] = _f64(sp.u[d]).ctypes.data
    s.w = _f64(sp.w).ctypes.data
    return s


def _rows(a):
    """View of a (3, N) array as three contiguous rows (no copy)."""
    a = _f64(a)
    return [a[0], a[1], a[2]]


# ------------------------------------------------------------------ API

def shape(order: int, a: float) -> float:
    return lib().orc_shape(order, a)


def gather(g: Grid, E, B, xi):
    Ef, Bf = _FieldPtrs(_rows(E)), _FieldPtrs(_rows(B))
    x = np.ascontiguousarray(xi, dtype=np.float64)
    Ep = np.zeros(3)
    Bp = np.zeros(3)
    lib().orc_gather(C.byref(g), Ef.ptr, Bf.ptr, x.ctypes.data, Ep.ctypes.data, Bp.ctypes.data)
    return Ep, Bp


def boris(q, m, dt, Ep, Bp, u):
    u = np.array(u, dtype=np.float64)
    Ep = np.ascontiguousarray(Ep, dtype=np.float64)
    Bp = np.ascontiguousarray(Bp, dtype=np.float64)
    lib().orc_boris(q, m, dt, Ep.ctypes.data, Bp.ctypes.data, u.ctypes.data)
    return u


def deposit(g: Grid, J, q, w, x0, x1, vy=0.0):
    """Adds one particle's Esirkepov current into J (3, N) in place."""
    Jf = _FieldPtrs(_rows(J))
    a0 = np.ascontiguousarray(x0, dtype=np.float64)
    a1 = np.ascontiguousarray(x1, dtype=np.float64)
    lib().orc_deposit(C.byref(g), Jf.ptr, q, w, a0.ctypes.data, a1.ctypes.data, vy)


def faraday(g: Grid, E, B, h):
    lib().orc_faraday(C.byref(g), _FieldPtrs(_rows(E)).ptr, _FieldPtrs(_rows(B)).ptr, h)


def ampere(g: Grid, E, B, J, dt):
    lib().orc_ampere(C.byref(g), _FieldPtrs(_rows(E)).ptr, _FieldPtrs(_rows(B)).ptr,
                     _FieldPtrs(_rows(J)).ptr, dt)


def fdtd_step(g: Grid, E, B, J):
    Ef, Bf, Jf = _FieldPtrs(_rows(E)), _FieldPtrs(_rows(B)), _FieldPtrs(_rows(J))
    lib().orc_fdtd_step(C.byref(g), Ef.ptr, Bf.ptr, Jf.ptr)


def wrap(x, L):
    return lib().orc_wrap(x, L)


def particles_step(g: Grid, E, B, J, species):
    """J is zeroed and filled; species arrays are updated in place."""
    Ef, Bf, Jf = _FieldPtrs(_rows(E)), _FieldPtrs(_rows(B)), _FieldPtrs(_rows(J))
    arr = (Species * len(species))(*[_species_struct(s) for s in species])
    lib().orc_particles_step(C.byref(g), Ef.ptr, Bf.ptr, Jf.ptr, arr, len(species))


def pic_step(g: Grid, E, B, J, species):
    Ef, Bf, Jf = _FieldPtrs(_rows(E)), _FieldPtrs(_rows(B)), _FieldPtrs(_rows(J))
    arr = (Species * len(species))(*[_species_struct(s) for s in species])
    lib().orc_pic_step(C.byref(g), Ef.ptr, Bf.ptr, Jf.ptr, arr, len(species))


def rho(g: Grid, species, ncells):
    out = np.zeros(ncells)
    for s in species:
        st = _species_struct(s)
        lib().orc_rho(C.byref(g), out.ctypes.data, C.byref(st))
    return out


def div_j(g: Grid, J, ncells):
    out = np.zeros(ncells)
    lib().orc_div_j(C.byref(g), _FieldPtrs(_rows(J)).ptr, out.ctypes.data)
    return out


def field_energy(g: Grid, E, B):
    return lib().orc_field_energy(C.byref(g), _FieldPtrs(_rows(E)).ptr, _FieldPtrs(_rows(B)).ptr)


def kinetic_energy(sp):
    st = _species_struct(sp)
    return lib().orc_kinetic_energy(C.byref(st))


def tile_keys(g: Grid, tile, sp):
    st = _species_struct(sp)
    t = np.ascontiguousarray(tile, dtype=np.int32)
    key = np.zeros(st.np, dtype=np.int32)
    lib().orc_tile_keys(C.byref(g), t.ctypes.data, C.byref(st), key.ctypes.data)
    return key


def cell_order_keys(g: Grid, tile, cbits, sp):
    """Within-tile cell-order sort keys (int64), see orc_cell_order_keys."""
    st = _species_struct(sp)
    t = np.ascontiguousarray(tile, dtype=np.int32)
    key = np.zeros(st.np, dtype=np.int64)
    lib().orc_cell_order_keys(C.byref(g), t.ctypes.data, int(cbits), C.byref(st), key.ctypes.data)
    return key


def tile_cell_keys(g: Grid, tile, cbits, sp):
    """Cell order without classes (int64 keys), see orc_tile_cell_keys."""
    st = _species_struct(sp)
    t = np.ascontiguousarray(tile, dtype=np.int32)
    key = np.zeros(st.np, dtype=np.int64)
    lib().orc_tile_cell_keys(C.byref(g), t.ctypes.data, int(cbits), C.byref(st), key.ctypes.data)
    return key


def stable_perm(key):
    key = np.ascontiguousarray(key, dtype=np.int64)
    perm = np.zeros(key.shape[0], dtype=np.int32)
    lib().orc_stable_perm(key.shape[0], key.ctypes.data, perm.ctypes.data)
    return perm


def quad_order(key, cbits):
    """Cell order with each tile's whole groups of four first (int32 perm)."""
    key = np.ascontiguousarray(key, dtype=np.int64)
    perm = np.zeros(key.shape[0], dtype=np.int32)
    lib().orc_quad_order(key.shape[0], key.ctypes.data, int(cbits), perm.ctypes.data)
    return perm


def stable_sort(key, nkeys):
    key = np.ascontiguousarray(key, dtype=np.int32)
    n = key.shape[0]
    perm = np.zeros(n, dtype=np.int32)
    count = np.zeros(nkeys, dtype=np.int32)
    offset = np.zeros(nkeys + 1, dtype=np.int32)
    lib().orc_stable_sort(n, key.ctypes.data, nkeys, perm.ctypes.data,
                          count.ctypes.data, offset.ctypes.data)
    return perm, count, offset


# ------------------------------------------------------------------ boundaries

def absorber(cells, sigma_max, power=3) -> Absorber:
    a = Absorber()
    a.cells, a.sigma_max, a.power = int(cells), float(sigma_max), int(power)
    return a


def absorber_sigma(a: Absorber, z, nz):
    return lib().orc_absorber_sigma(C.byref(a), float(z), float(nz))


def fdtd_step_absorb(g: Grid, E, B, J, a: Absorber, zoff=0.0):
    Ef, Bf, Jf = _FieldPtrs(_rows(E)), _FieldPtrs(_rows(B)), _FieldPtrs(_rows(J))
    lib().orc_fdtd_step_absorb(C.byref(g), Ef.ptr, Bf.ptr, Jf.ptr, C.byref(a), float(zoff))


def antenna(k, E0, omega, waist, x0, y0, t0, tau) -> Antenna:
    an = Antenna()
    an.k, an.E0, an.omega, an.waist = int(k), float(E0), float(omega), float(waist)
    an.x0, an.y0, an.t0, an.tau = float(x0), float(y0), float(t0), float(tau)
    return an


def antenna_add(g: Grid, J, an: Antenna, t):
    lib().orc_antenna_add(C.byref(g), _FieldPtrs(_rows(J)).ptr, C.byref(an), float(t))


def window_shift_fields(g: Grid, E, B):
    lib().orc_window_shift_fields(C.byref(g), _FieldPtrs(_rows(E)).ptr, _FieldPtrs(_rows(B)).ptr)


def window_shift_particles(g: Grid, sp):
    """Shifts and compacts ``sp`` (x, u, w arrays of capacity >= np) in place;
    returns the new count.  ``sp.np`` (if present) is not changed."""
    st = _species_struct(sp)
    return int(lib().orc_window_shift_particles(C.byref(g), C.byref(st)))


# ------------------------------------------------------------------ electrostatic

def poisson_periodic(g: Grid, rho):
    """phi solving the discrete periodic Poisson equation div grad phi =
    -(rho - mean rho) with the Yee differences (the 7-point Laplacian; 5
    points in 2D), mean of phi zero.  Exact, by the discrete Fourier
    transform: each mode of the Laplacian has eigenvalue -sum_d (2 - 2
    cos(2 pi k_d / n_d)) / dx_d^2."""
    n = [int(g.n[d]) for d in range(3)]
    r = np.asarray(rho, dtype=np.float64).reshape(n[2], n[1], n[0])
    rh = np.fft.fftn(r - r.mean())
    lam = np.zeros((n[2], n[1], n[0]))
    for d, ax in ((0, 2), (1, 1), (2, 0)):
        if g.dim == 2 and d == 1:
            continue
        k = np.arange(n[d])
        l1 = (2.0 - 2.0 * np.cos(2.0 * np.pi * k / n[d])) / (g.dx[d] ** 2)
        shape = [1, 1, 1]
        shape[ax] = n[d]
        lam = lam + l1.reshape(shape)
    lam[0, 0, 0] = 1.0
    ph = rh / lam
    ph[0, 0, 0] = 0.0
    return np.ascontiguousarray(np.real(np.fft.ifftn(ph)).reshape(-1))


def es_field(g: Grid, phi):
    E = np.zeros((3, int(np.prod([g.n[d] for d in range(3)]))))
    lib().orc_es_field(C.byref(g), _f64(np.ascontiguousarray(phi)).ctypes.data,
                       _FieldPtrs(_rows(E)).ptr)
    return E


def es_particles_step(g: Grid, E, species):
    Ef = _FieldPtrs(_rows(E))
    arr = (Species * len(species))(*[_species_struct(s) for s in species])
    lib().orc_es_particles_step(C.byref(g), Ef.ptr, arr, len(species))


def es_step(g: Grid, species, ncells):
    """One electrostatic step: rho of the species, Poisson, E = -grad phi,
    particle update.  Returns (rho, phi, E) of the step's start."""
    r = rho(g, species, ncells)
    phi = poisson_periodic(g, r)
    E = es_field(g, phi)
    es_particles_step(g, E, species)
    return r, phi, E


# ------------------------------------------------------------------ variants

def vay(q, m, dt, Ep, Bp, u):
    u = np.array(u, dtype=np.float64)
    Ep = np.ascontiguousarray(Ep, dtype=np.float64)
    Bp = np.ascontiguousarray(Bp, dtype=np.float64)
    lib().orc_vay(q, m, dt, Ep.ctypes.data, Bp.ctypes.data, u.ctypes.data)
    return u


def gather_galerkin(g: Grid, E, B, xi):
    Ef, Bf = _FieldPtrs(_rows(E)), _FieldPtrs(_rows(B))
    x = np.ascontiguousarray(xi, dtype=np.float64)
    Ep, Bp = np.zeros(3), np.zeros(3)
    lib().orc_gather_galerkin(C.byref(g), Ef.ptr, Bf.ptr, x.ctypes.data, Ep.ctypes.data,
                              Bp.ctypes.data)
    return Ep, Bp


def particles_step_opts(g: Grid, E, B, J, species, pusher=0, gather=0):
    Ef, Bf, Jf = _FieldPtrs(_rows(E)), _FieldPtrs(_rows(B)), _FieldPtrs(_rows(J))
    arr = (Species * len(species))(*[_species_struct(s) for s in species])
    lib().orc_particles_step_opts(C.byref(g), Ef.ptr, Bf.ptr, Jf.ptr, arr, len(species),
                                  int(pusher), int(gather))


def slice_moments(g: Grid, sp, zoff=0):
    """(n_z, 5): per z layer sum w, w u_x, w u_y, w u_z, w m (gamma - 1)."""
    out = np.zeros(5 * int(g.n[2]))
    st = _species_struct(sp)
    lib().orc_slice_moments(C.byref(g), C.byref(st), int(zoff), out.ctypes.data)
    return out.reshape(-1, 5)


def rank_major(key, cbits, rbits=4):
    """Rank-major within-tile order of (tile, cell) keys (int64 array)."""
    k = np.ascontiguousarray(key, dtype=np.int64)
    perm = np.zeros(k.shape[0], dtype=np.int32)
    lib().orc_rank_major(k.shape[0], k.ctypes.data, int(cbits), int(rbits), perm.ctypes.data)
    return perm

