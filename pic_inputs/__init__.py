"""Seeded synthetic inputs for the PIC hot path, shared by the GPU path's tests
and benchmark and by the CPU oracle's tests.

This module holds no arithmetic of the method itself (no shape factor, no
push, no deposit, no field solve): only the initial conditions -- box
geometry, particle positions, momenta and weights, and initial fields -- each
drawn from a seeded ``torch.Generator`` on the requested device.  The recipe
of every workload is stated at its builder.

Normalised units: c = eps0 = mu0 = 1, cell size 1, time in cell/c.  Particle
positions are kept in cell units.  In-cell offsets are drawn as integer
multiples of 2**-24, so that ``x = cell + offset`` is exact in FP64 and the
split representation (int32 cell, FP32 offset) holds the very same position;
momenta, weights and fields are rounded through FP32 for the same reason.
The FP64 and split-precision runs therefore start from bit-identical states.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import numpy as np
import torch

DT3 = 0.99 / math.sqrt(3.0)      # CFL 0.99, cubic cells
DT2 = 0.99 / math.sqrt(2.0)      # CFL 0.99, square cells (x-z plane)
LAMBDA0 = 20.0                   # laser wavelength in cells
OMEGA0 = 2.0 * math.pi / LAMBDA0 # = k0 (c = 1)
N_CRIT = OMEGA0 ** 2             # critical density in these units
SEED0 = 2303128730
M_ION = 1836.0


@dataclass
class Box:
    dim: int                       # 2 (x-z plane) or 3
    n: Tuple[int, int, int]        # cells (n[1] == 1 in 2D)
    dt: float
    order: int                     # shape order 1..3
    tile: Tuple[int, int, int] = (8, 8, 8)
    dx: Tuple[float, float, float] = (1.0, 1.0, 1.0)

    @property
    def ncells(self) -> int:
        return self.n[0] * self.n[1] * self.n[2]

    @property
    def ntiles(self) -> int:
        t = 1
        for d in range(3):
            t *= -(-self.n[d] // self.tile[d])
        return t


@dataclass
class Particles:
    """One species in one box; arrays are torch tensors on one device."""
    q: float
    m: float
    x: torch.Tensor                # (3, np) float64, cell units, [0, n)
    u: torch.Tensor                # (3, np) float64, u = gamma v
    w: torch.Tensor                # (np,) float64
    cell: torch.Tensor             # (np,) int32 linear cell id in the box
    off: torch.Tensor              # (3, np) float32 in-cell offsets in [0, 1)
    box: int = 0

    @property
    def np(self) -> int:
        return int(self.w.shape[0])

    def to(self, device) -> "Particles":
        return Particles(self.q, self.m, self.x.to(device), self.u.to(device),
                         self.w.to(device), self.cell.to(device),
                         self.off.to(device), self.box)

    def numpy(self):
        """Independent numpy float64 copies of x, u, w (what the oracle
        consumes and updates in place)."""
        return SimpleSpecies(self.q, self.m,
                             np.array(self.x.cpu().numpy(), dtype=np.float64, order="C", copy=True),
                             np.array(self.u.cpu().numpy(), dtype=np.float64, order="C", copy=True),
                             np.array(self.w.cpu().numpy(), dtype=np.float64, order="C", copy=True))

    def select(self, idx: torch.Tensor) -> "Particles":
        return Particles(self.q, self.m, self.x[:, idx].contiguous(),
                         self.u[:, idx].contiguous(), self.w[idx].contiguous(),
                         self.cell[idx].contiguous(), self.off[:, idx].contiguous(),
                         self.box)


@dataclass
class SimpleSpecies:
    q: float
    m: float
    x: np.ndarray
    u: np.ndarray
    w: np.ndarray


@dataclass
class Workload:
    name: str
    boxes: List[Box]
    species: List[Particles]
    E: List[torch.Tensor]          # per box, (3, ncells) float64
    B: List[torch.Tensor]
    steps: int = 10
    notes: str = ""

    @property
    def np_total(self) -> int:
        return sum(s.np for s in self.species)


# --------------------------------------------------------------- primitives

def _gen(seed: int, device) -> torch.Generator:
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    return g


def _round32(t: torch.Tensor) -> torch.Tensor:
    return t.to(torch.float32).to(torch.float64)


def _offsets(n: int, g, device) -> torch.Tensor:
    """Uniform in-cell offsets on the 2**-24 lattice inside [0, 1)."""
    k = torch.randint(0, 1 << 24, (n,), generator=g, device=device, dtype=torch.int64)
    return k.to(torch.float64) * (2.0 ** -24)


def _cell_coords(box: Box, cell: torch.Tensor):
    cx = cell % box.n[0]
    cy = (cell // box.n[0]) % box.n[1]
    cz = cell // (box.n[0] * box.n[1])
    return cx, cy, cz


def particles_in_cells(box: Box, cells: torch.Tensor, ppc, weight, q, m,
                       u_th: float, seed: int, device, box_index: int = 0) -> Particles:
    """``ppc`` particles per listed cell (cell-major order), uniform inside the
    cell; Maxwellian momenta of spread ``u_th`` per component (cold if 0);
    ``weight`` is a scalar or one value per listed cell.  ``ppc`` may be a
    scalar or one count per listed cell."""
    g = _gen(seed, device)
    cells = cells.to(device=device, dtype=torch.int64)
    if isinstance(ppc, torch.Tensor):
        counts = ppc.to(device=device, dtype=torch.int64)
        cell = torch.repeat_interleave(cells, counts)
        wcell = weight if not isinstance(weight, torch.Tensor) else \
            torch.repeat_interleave(weight.to(device), counts)
    else:
        cell = torch.repeat_interleave(cells, int(ppc))
        wcell = weight if not isinstance(weight, torch.Tensor) else \
            torch.repeat_interleave(weight.to(device), int(ppc))
    npart = cell.shape[0]
    cx, cy, cz = _cell_coords(box, cell)
    off = torch.stack([_offsets(npart, g, device),
                       _offsets(npart, g, device) if box.dim == 3 else torch.zeros(npart, dtype=torch.float64, device=device),
                       _offsets(npart, g, device)])
    x = torch.stack([cx.to(torch.float64), cy.to(torch.float64), cz.to(torch.float64)]) + off
    if u_th > 0:
        u = _round32(torch.randn((3, npart), generator=g, device=device, dtype=torch.float64) * u_th)
    else:
        u = torch.zeros((3, npart), dtype=torch.float64, device=device)
    if isinstance(wcell, torch.Tensor):
        w = _round32(wcell.to(torch.float64))
    else:
        w = torch.full((npart,), float(np.float32(wcell)), dtype=torch.float64, device=device)
    return Particles(q, m, x.contiguous(), u.contiguous(), w.contiguous(),
                     cell.to(torch.int32).contiguous(), off.to(torch.float32).contiguous(),
                     box_index)


def zero_fields(box: Box, device):
    z = lambda: torch.zeros((3, box.ncells), dtype=torch.float64, device=device)
    return z(), z()


def _stagger_coords(box: Box, comp: int, kind: str, device):
    """Physical coordinates (cell units) of a field component's Yee points."""
    i = torch.arange(box.n[0], dtype=torch.float64, device=device)
    j = torch.arange(box.n[1], dtype=torch.float64, device=device)
    k = torch.arange(box.n[2], dtype=torch.float64, device=device)
    sh = [0.0, 0.0, 0.0]
    for d in range(3):
        on = (d == comp) if kind == "E" else (d != comp)
        sh[d] = 0.5 if on else 0.0
    if box.dim == 2:
        sh[1] = 0.0
    Z, Y, X = torch.meshgrid(k + sh[2], j + sh[1], i + sh[0], indexing="ij")
    return X.reshape(-1), Y.reshape(-1), Z.reshape(-1)


def fourier_fields(box: Box, modes: int, amp: float, seed: int, device):
    """Smooth periodic fields: a few random Fourier modes per component,
    sampled at each component's own Yee points, rounded through FP32."""
    g = _gen(seed, "cpu")
    E = torch.zeros((3, box.ncells), dtype=torch.float64, device=device)
    B = torch.zeros((3, box.ncells), dtype=torch.float64, device=device)
    for F, kind in ((E, "E"), (B, "B")):
        for c in range(3):
            X, Y, Z = _stagger_coords(box, c, kind, device)
            for _ in range(modes):
                kv = torch.randint(-2, 3, (3,), generator=g)
                if box.dim == 2:
                    kv[1] = 0
                a = float(torch.rand((), generator=g, dtype=torch.float64)) * amp
                ph = float(torch.rand((), generator=g, dtype=torch.float64)) * 2 * math.pi
                arg = 2 * math.pi * (kv[0] * X / box.n[0] + kv[1] * Y / box.n[1] + kv[2] * Z / box.n[2])
                F[c] += a * torch.sin(arg + ph)
    return _round32(E), _round32(B)


def laser_fields(box: Box, a0: float, waist: float, length: float, z0: float,
                 center: Tuple[float, float], device):
    """Gaussian laser pulse, Ex-polarised, propagating along +z, focused at
    its centroid (flat phase): Ex = E0 exp(-r^2/w0^2) exp(-(z-z0)^2/L^2)
    cos(k0 (z-z0)), By = Ex taken at By's Yee points, E0 = a0 * omega0."""
    E = torch.zeros((3, box.ncells), dtype=torch.float64, device=device)
    B = torch.zeros((3, box.ncells), dtype=torch.float64, device=device)
    E0 = a0 * OMEGA0

    def profile(X, Y, Z):
        r2 = (X - center[0]) ** 2 + ((Y - center[1]) ** 2 if box.dim == 3 else 0.0)
        return E0 * torch.exp(-r2 / waist ** 2) * torch.exp(-((Z - z0) / length) ** 2) * \
            torch.cos(OMEGA0 * (Z - z0))

    # The position of cell centre vs node: profiles are evaluated at the
    # physical location of each Yee point, coordinates in cell units.
    X, Y, Z = _stagger_coords(box, 0, "E", device)
    E[0] = profile(X, Y, Z)
    X, Y, Z = _stagger_coords(box, 1, "B", device)
    B[1] = profile(X, Y, Z)
    return _round32(E), _round32(B)


def ramp_density(zc: torch.Tensor, n0: float, z_start=120.0, z_plateau=220.0):
    """Vacuum below z_start, linear ramp to n0 at z_plateau, then flat."""
    return n0 * torch.clamp((zc - z_start) / (z_plateau - z_start), 0.0, 1.0)


# --------------------------------------------------------------- workloads

def uniform_box(n=(32, 32, 32), ppc=8, n0=0.01, u_th=0.01, order=1, seed=SEED0,
                device="cpu", tile=(8, 8, 8), fields: Optional[str] = None,
                species=("e",), dim=3) -> Workload:
    """Periodic box, ``ppc`` particles in every cell at uniform positions,
    Maxwellian momenta u_th, weight n0*dV/ppc.  fields=None: E = B = 0
    (immobile neutralising background implied, not deposited);
    fields="fourier": three random smooth modes per component."""
    dt = DT3 if dim == 3 else DT2
    nn = tuple(n) if dim == 3 else (n[0], 1, n[2])
    box = Box(dim, nn, dt, order, tuple(tile) if dim == 3 else (tile[0], 1, tile[2]))
    cells = torch.arange(box.ncells, dtype=torch.int64)
    sps = []
    for si, s in enumerate(species):
        q, m = (-1.0, 1.0) if s == "e" else (1.0, M_ION)
        sps.append(particles_in_cells(box, cells, ppc, n0 / ppc, q, m, u_th,
                                      seed + 100 * si, device))
    if fields == "fourier":
        E, B = fourier_fields(box, 3, 0.01, seed + 7, device)
    else:
        E, B = zero_fields(box, device)
    return Workload("uniform", [box], sps, [E], [B], 10)


def c1(device="cpu", fields=None) -> Workload:
    """32^3 periodic, 8 electrons/cell, u_th = 0.01, n0 = 0.01, order 1,
    FP64, CFL 0.99, 10 steps, E = B = 0 (fields="fourier" gives the variant
    with seeded smooth fields)."""
    w = uniform_box((32, 32, 32), 8, 0.01, 0.01, 1, SEED0 + 0, device, fields=fields)
    w.name = "c1_32cube_ppc8_order1" + ("_fourier" if fields else "")
    return w


def c3(device="cpu", fields=None) -> Workload:
    """The inputs of c1 with order-3 shapes (split-precision form)."""
    w = uniform_box((32, 32, 32), 8, 0.01, 0.01, 3, SEED0 + 0, device, fields=fields)
    w.name = "c3_32cube_ppc8_order3" + ("_fourier" if fields else "")
    return w


def lwfa_box(n, ppc, order, a0, species=("e",), seed=SEED0 + 1, device="cpu",
             tile=(8, 8, 8), z_slab: Optional[Tuple[int, int]] = None,
             u_th: float = 0.01) -> Workload:
    """Laser-wakefield box: laser (lambda = 20 cells, waist 16, length 20,
    centroid z0 = 60, centred transversely) in vacuum below z = 120, plasma
    ramp 120 -> 220 then n0 = 1e-3 n_c, ``ppc`` particles per cell wherever
    n > 0 (weight n dV / ppc).  The plasma temperature is not given by the
    workload description; electrons get a thermal spread u_th (default
    0.01 c, as the uniform boxes) and ions the same temperature
    (u_th / sqrt(m_i/m_e)), so every particle moves from the first step.
    ``z_slab`` restricts the particles to cell layers [z_lo, z_hi) (bounded
    samples of the same workload)."""
    box = Box(3, tuple(n), DT3, order, tuple(tile))
    n0 = 1e-3 * N_CRIT
    k = torch.arange(box.n[2], dtype=torch.float64)
    dens = ramp_density(k + 0.5, n0)
    layers = torch.nonzero(dens > 0).flatten()
    if z_slab is not None:
        layers = layers[(layers >= z_slab[0]) & (layers < z_slab[1])]
    per_layer = box.n[0] * box.n[1]
    cells = (layers[:, None] * per_layer + torch.arange(per_layer)[None, :]).reshape(-1)
    wcell = torch.repeat_interleave(dens[layers] / ppc, per_layer)
    sps = []
    for si, s in enumerate(species):
        q, m = (-1.0, 1.0) if s == "e" else (1.0, M_ION)
        sps.append(particles_in_cells(box, cells, ppc, wcell, q, m, u_th / math.sqrt(m),
                                      seed + 100 * si, device))
    E, B = laser_fields(box, a0, 16.0, 20.0, 60.0, (box.n[0] / 2, box.n[1] / 2), device)
    return Workload("lwfa", [box], sps, [E], [B], 200)


def c2(device="cpu", scale=1) -> Workload:
    """128x128x1024, 2 e-/cell, order 2, a0 = 2, FP64, 200 steps.  ``scale``
    > 1 divides the transverse size (small copies for tests)."""
    n = (128 // scale, 128 // scale, 1024)
    w = lwfa_box(n, 2, 2, 2.0, ("e",), SEED0 + 1, device)
    w.name = f"c2_lwfa_{n[0]}x{n[1]}x{n[2]}_ppc2_order2"
    return w


def c5(device="cpu", scale=1, z_slab=None) -> Workload:
    """256x256x2048, electrons + ions (m = 1836), 4 each per cell co-located
    in cell (independent offsets), order 3, a0 = 4, 500 steps."""
    n = (256 // scale, 256 // scale, 2048)
    w = lwfa_box(n, 4, 3, 4.0, ("e", "i"), SEED0 + 4, device, z_slab=z_slab)
    w.name = f"c5_lwfa_{n[0]}x{n[1]}x{n[2]}_2sp_ppc4_order3"
    w.steps = 500
    return w


def c4(device="cpu", nboxes=64, l_range=(64, 512), big=(256, 256, 256),
       mean_tile=4096, sigma=1.5, shell_radius=64.0, seed=SEED0 + 3) -> Workload:
    """Batched form: ``nboxes`` independent square 2D x-z boxes with side
    L ~ U{64..512} and ppc ~ U{1..16} (u_th 0.01, n0 0.01, order 2, CFL 0.99
    in 2D), plus one 3D box with 8^3 tiles whose particle counts are
    round(LogNormal(mu, sigma)) with mean ``mean_tile``, placed so the
    largest counts sit on a spherical shell of radius ``shell_radius``
    around the box centre (a bubble-like spike); particles uniform inside
    their tile.  Momenta u_th = 0.01; weight n0 dV * 8 / (mean ppc)."""
    g = _gen(seed, "cpu")
    boxes, sps, Es, Bs = [], [], [], []
    order = 2
    for b in range(nboxes):
        L = int(torch.randint(l_range[0], l_range[1] + 1, (1,), generator=g))
        ppc = int(torch.randint(1, 17, (1,), generator=g))
        box = Box(2, (L, 1, L), DT2, order, (8, 1, 8))
        cells = torch.arange(box.ncells, dtype=torch.int64)
        sps.append(particles_in_cells(box, cells, ppc, 0.01 / ppc, -1.0, 1.0, 0.01,
                                      seed + 1000 + b, device, box_index=b))
        E, B = zero_fields(box, device)
        boxes.append(box); Es.append(E); Bs.append(B)
    box3 = Box(3, tuple(big), DT3, order, (8, 8, 8))
    nt = [box3.n[d] // 8 for d in range(3)]
    ntiles = nt[0] * nt[1] * nt[2]
    mu = math.log(mean_tile) - 0.5 * sigma * sigma
    counts = torch.round(torch.exp(mu + sigma * torch.randn(ntiles, generator=g, dtype=torch.float64)))
    counts = torch.sort(counts, descending=True).values.to(torch.int64)
    t = torch.arange(ntiles)
    tx, ty, tz = t % nt[0], (t // nt[0]) % nt[1], t // (nt[0] * nt[1])
    ctr = [box3.n[d] / 2 for d in range(3)]
    dist = torch.sqrt(((tx * 8 + 4 - ctr[0]) ** 2 + (ty * 8 + 4 - ctr[1]) ** 2 +
                       (tz * 8 + 4 - ctr[2]) ** 2).to(torch.float64))
    order_t = torch.argsort(torch.abs(dist - shell_radius), stable=True)
    tile_counts = torch.zeros(ntiles, dtype=torch.int64)
    tile_counts[order_t] = counts
    # Particles uniform inside each tile: pick a cell of the tile uniformly,
    # then a uniform offset inside the cell.
    gd = _gen(seed + 2000, device)
    tot = int(tile_counts.sum())
    tid = torch.repeat_interleave(t.to(device), tile_counts.to(device))
    lc = torch.randint(0, 512, (tot,), generator=gd, device=device)
    ttx, tty, ttz = tid % nt[0], (tid // nt[0]) % nt[1], tid // (nt[0] * nt[1])
    cx = ttx * 8 + lc % 8
    cy = tty * 8 + (lc // 8) % 8
    cz = ttz * 8 + lc // 64
    cell = cx + box3.n[0] * (cy + box3.n[1] * cz)
    del lc, ttx, tty, ttz, cx, cy, cz, tid
    w3 = 0.01 * 512 / mean_tile
    sp3 = particles_in_cells(box3, cell, 1, w3, -1.0, 1.0, 0.01, seed + 3000, device,
                             box_index=nboxes)
    del cell
    E, B = zero_fields(box3, device)
    boxes.append(box3); sps.append(sp3); Es.append(E); Bs.append(B)
    return Workload("c4_batched_64x2d_plus_256cube_lognormal", boxes, sps, Es, Bs, 10)


def particles_from_positions(box: Box, x, u, w, q: float, m: float, device="cpu",
                             box_index: int = 0) -> Particles:
    """A species from explicit positions (cell units, (3, np), each in-cell
    offset on the 2**-24 lattice so that the split form holds it exactly),
    momenta (3, np) and weights (np,); for hand-built edge cases."""
    x = torch.as_tensor(np.asarray(x, dtype=np.float64), device=device).clone()
    u = torch.as_tensor(np.asarray(u, dtype=np.float64), device=device).clone()
    w = torch.as_tensor(np.asarray(w, dtype=np.float64), device=device).clone()
    if box.dim == 2:
        x[1] = 0.0
    c = torch.floor(x)
    off = x - c
    if not bool(torch.all(off * (1 << 24) == torch.round(off * (1 << 24)))):
        raise ValueError("offsets must lie on the 2**-24 lattice")
    ci = c.to(torch.int64)
    cell = ci[0] + box.n[0] * (ci[1] + box.n[1] * ci[2])
    return Particles(q, m, x.contiguous(), u.contiguous(), w.contiguous(),
                     cell.to(torch.int32).contiguous(), off.to(torch.float32).contiguous(),
                     box_index)
