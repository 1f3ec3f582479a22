"""Pins of the oracle's whole particle step and of its energy diagnostics.

``orc_particles_step`` is driven through whole steps in fields whose exact
discrete trajectories are known in closed form, computed here without any
of the oracle's arithmetic:

* free streaming (E = B = 0): every step moves a particle by exactly
  dt u / (gamma dx_d) along each axis, wrapped periodically, with
  anisotropic cells and relativistic momenta;
* uniform B along z: the Boris step rotates u by theta = 2 atan(|q| B dt /
  (2 m gamma)) per step, so x^n = x^0 + sum_{k=1..n} dt R(k theta) u^(-1/2)
  / (gamma dx): the chord of step k uses the momentum AFTER the k-th push
  (u^(n+1/2)), and the points lie on a circle of radius
  dt v_perp / (2 sin(theta / 2));
* uniform E perpendicular to B (|E| < |B|): the scheme's exact fixed point
  u* = (E/B) sqrt((1 + h^2 E^2) / (1 - E^2/B^2)) along E x B stays put and
  x advances by dt v* per step;
* a field linear in z: the gathered value is exact (first moment of the
  B-splines), so the momentum change of one step fixes WHERE the gather
  happened (x^n, not x^(n+1)).

Energies: uniform fields and a single Fourier mode have closed-form sums;
the kinetic energy m (gamma - 1) is checked on exact Pythagorean momenta and
against its series at small |u|.
"""
import math

import numpy as np
import pytest

import oracle
import pic_inputs as pi


class _Sp:
    def __init__(self, q, m, x, u, w):
        self.q, self.m = q, m
        # own copies: the oracle updates them in place
        self.x = np.array(x, dtype=np.float64, order="C", copy=True)
        self.u = np.array(u, dtype=np.float64, order="C", copy=True)
        self.w = np.array(w, dtype=np.float64, order="C", copy=True)


def _zeros(n):
    return np.zeros((3, int(np.prod(n))))


def _run(g, n, E, B, sp, steps):
    """Positions after every step (steps+1, 3, np) and final u."""
    J = _zeros(n)
    xs = [sp.x.copy()]
    for _ in range(steps):
        oracle.particles_step(g, E, B, J, [sp])
        xs.append(sp.x.copy())
    return np.array(xs)


def _fold(d, L):
    L = np.asarray(L, dtype=np.float64).reshape(3, 1)
    return d - L * np.round(d / L)


@pytest.mark.parametrize("dim", (3, 2))
@pytest.mark.parametrize("order", (1, 2, 3))
def test_free_streaming_advance(dim, order):
    n = (9, 7, 11) if dim == 3 else (9, 1, 11)
    dx = (1.0, 0.7, 1.3) if dim == 3 else (1.0, 1.0, 1.3)
    inv = sum(1.0 / d ** 2 for k, d in enumerate(dx) if not (dim == 2 and k == 1))
    dt = 0.95 / math.sqrt(inv)
    g = oracle.make_grid(dim, n, dx, dt, order)
    rng = np.random.default_rng(5)
    npart = 40
    x = np.stack([rng.uniform(0, n[0], npart), rng.uniform(0, n[1], npart) if dim == 3
                  else np.zeros(npart), rng.uniform(0, n[2], npart)])
    # near the seams, so that wraps happen in both directions
    x[0, :5] = n[0] - 1e-3
    x[2, 5:10] = 1e-3
    u = rng.normal(0.0, 1.5, (3, npart))          # relativistic: gamma up to ~4
    u[:, 5:10] = -np.abs(u[:, 5:10])
    sp = _Sp(-1.0, 1.0, x, u, np.full(npart, 0.1))
    steps = 6
    xs = _run(g, n, _zeros(n), _zeros(n), sp, steps)
    gam = np.sqrt(1.0 + np.sum(u * u, axis=0))
    step = np.array([dt * u[d] / (gam * dx[d]) for d in range(3)])
    if dim == 2:
        step[1] = 0.0
    L = np.array(n, dtype=np.float64)
    for k in range(steps + 1):
        expect = np.mod(x + k * step, L[:, None])
        d = _fold(xs[k] - expect, n)
        assert np.max(np.abs(d)) < 1e-12, (k, np.max(np.abs(d)))
        assert np.all(xs[k] >= 0.0) and np.all(xs[k] < L[:, None])
    np.testing.assert_array_equal(sp.u, u)        # no field, no change


@pytest.mark.parametrize("q,m", ((-1.0, 1.0), (1.0, 1836.0), (1.0, 2.0)))
def test_gyration_positions_closed_form(q, m):
    n = (40, 40, 8)
    dx = (1.0, 1.0, 1.0)
    dt = pi.DT3
    g = oracle.make_grid(3, n, dx, dt, 2)
    Bz = 0.35 * m
    B = _zeros(n)
    B[2][:] = Bz
    u0 = np.array([0.9, -0.4, 0.25])
    gam = math.sqrt(1.0 + u0 @ u0)
    theta = 2.0 * math.atan(abs(q) * Bz * dt / (2.0 * m * gam))
    sgn = -math.copysign(1.0, q)           # dot(u) = (q/m) u x B / gamma: clockwise for q > 0
    x0 = np.array([20.3, 19.6, 4.1])
    sp = _Sp(q, m, x0[:, None], u0[:, None], np.array([1.0]))
    steps = 25
    xs = _run(g, n, _zeros(n), B, sp, steps)[:, :, 0]
    expect = x0.copy()
    pts = [expect.copy()]
    for k in range(1, steps + 1):
        a = sgn * k * theta
        uk = np.array([math.cos(a) * u0[0] - math.sin(a) * u0[1],
                       math.sin(a) * u0[0] + math.cos(a) * u0[1], u0[2]])
        expect = expect + dt * uk / gam
        pts.append(expect.copy())
        d = _fold((xs[k] - np.mod(expect, n))[:, None], n)
        assert np.max(np.abs(d)) < 1e-11, (k, d.ravel())
    # the in-plane points lie on one circle of radius dt v_perp / (2 sin(theta/2))
    vperp = math.hypot(u0[0], u0[1]) / gam
    R = dt * vperp / (2.0 * math.sin(theta / 2.0))
    P = np.array(pts)[:, :2]
    # center from the first three points (circumcircle)
    (ax, ay), (bx, by), (cx, cy) = P[0], P[1], P[2]
    dd = 2.0 * (ax * (by - cy) + bx * (cy - ay) + cx * (ay - by))
    ux = ((ax * ax + ay * ay) * (by - cy) + (bx * bx + by * by) * (cy - ay) +
          (cx * cx + cy * cy) * (ay - by)) / dd
    uy = ((ax * ax + ay * ay) * (cx - bx) + (bx * bx + by * by) * (ax - cx) +
          (cx * cx + cy * cy) * (bx - ax)) / dd
    r = np.hypot(P[:, 0] - ux, P[:, 1] - uy)
    assert np.max(np.abs(r - R)) < 1e-10 * max(R, 1.0)


@pytest.mark.parametrize("q", (-1.0, 1.0))
def test_exb_drift_positions(q):
    n = (16, 64, 16)
    dt = pi.DT3
    m = 1.0
    g = oracle.make_grid(3, n, (1.0, 1.0, 1.0), dt, 3)
    Ex, Bz = 0.12, 0.3
    E = _zeros(n)
    E[0][:] = Ex
    B = _zeros(n)
    B[2][:] = Bz
    h = q * dt / (2.0 * m)
    U = (Ex / Bz) * math.sqrt((1.0 + h * h * Ex * Ex) / (1.0 - Ex * Ex / (Bz * Bz)))
    # E x B = x^ x z^ = -y^
    u0 = np.array([0.0, -U, 0.0])
    x0 = np.array([3.25, 10.5, 7.75])
    sp = _Sp(q, m, x0[:, None], u0[:, None], np.array([1.0]))
    steps = 40
    xs = _run(g, n, E, B, sp, steps)[:, :, 0]
    assert np.max(np.abs(sp.u[:, 0] - u0)) < 1e-13
    v = U / math.sqrt(1.0 + U * U)
    for k in range(steps + 1):
        expect = np.mod(x0 + k * dt * np.array([0.0, -v, 0.0]), n)
        d = _fold((xs[k] - expect)[:, None], n)
        assert np.max(np.abs(d)) < 1e-11, (k, d.ravel())


@pytest.mark.parametrize("dim", (3, 2))
@pytest.mark.parametrize("order", (1, 2, 3))
def test_gather_happens_at_old_position(dim, order):
    n = (6, 5, 24) if dim == 3 else (6, 1, 24)
    dt = pi.DT3 if dim == 3 else pi.DT2
    g = oracle.make_grid(dim, n, (1.0, 1.0, 1.0), dt, order)
    a, b = 0.02, 0.01
    E = _zeros(n)
    k = np.arange(n[2], dtype=np.float64)
    # Ex at (i+1/2, j, k): linear in the node index k along z
    E[0] = np.broadcast_to((a + b * k)[:, None, None], (n[2], n[1], n[0])).ravel()
    q, m = -1.0, 1.0
    z0 = 9.37
    uz = 3.0                                   # moves ~0.55 cell per step along z
    x0 = np.array([2.5, 2.0 if dim == 3 else 0.0, z0])
    u0 = np.array([0.0, 0.0, uz])
    sp = _Sp(q, m, x0[:, None], u0[:, None], np.array([1.0]))
    J = _zeros(n)
    oracle.particles_step(g, E, _zeros(n), J, [sp])
    du = sp.u[0, 0] - u0[0]
    expect = (q / m) * dt * (a + b * z0)
    assert abs(du - expect) < 1e-15
    # the new position would give a clearly different kick
    gam = math.sqrt(1.0 + sp.u[:, 0] @ sp.u[:, 0])
    z1 = z0 + dt * sp.u[2, 0] / gam
    assert abs((q / m) * dt * (a + b * z1) - expect) > 1e-4


# ------------------------------------------------------------------ energies

def test_field_energy_uniform_fields():
    n = (5, 4, 3)
    dx = (0.5, 1.25, 2.0)
    g = oracle.make_grid(3, n, dx, 0.1, 1)
    ncell = 60
    vals = [0.3, -1.5, 2.0, 0.25, -0.75, 1.0]
    E = np.array([np.full(ncell, v) for v in vals[:3]])
    B = np.array([np.full(ncell, v) for v in vals[3:]])
    dV = 0.5 * 1.25 * 2.0
    expect = 0.5 * sum(v * v for v in vals) * ncell * dV
    assert abs(oracle.field_energy(g, E, B) - expect) < 1e-14 * expect
    # E and B enter alike, each component once
    assert abs(oracle.field_energy(g, B, E) - expect) < 1e-14 * expect
    Z = np.zeros_like(E)
    eE = 0.5 * sum(v * v for v in vals[:3]) * ncell * dV
    assert abs(oracle.field_energy(g, E, Z) - eE) < 1e-14 * eE


@pytest.mark.parametrize("mode", (1, 3))
def test_field_energy_fourier_mode(mode):
    # A sin(2 pi m i / N) summed in square over whole periods is A^2 N / 2.
    n = (16, 6, 10)
    g = oracle.make_grid(3, n, (1.0, 1.0, 1.0), 0.1, 2)
    i = np.arange(n[0])
    A = 0.7
    prof = A * np.sin(2 * math.pi * mode * i / n[0])
    By = np.broadcast_to(prof[None, None, :], (n[2], n[1], n[0])).ravel()
    E = np.zeros((3, 960))
    B = np.zeros((3, 960))
    B[1] = By
    expect = 0.5 * A * A * (n[0] / 2.0) * n[1] * n[2]
    assert abs(oracle.field_energy(g, E, B) - expect) < 1e-13 * expect


def test_kinetic_energy_exact_momenta():
    # Pythagorean momenta: |u| = 3/4 -> gamma = 5/4; |u| = 12/5 -> 13/5;
    # u = (2, 3, 6): |u| = 7 -> gamma = sqrt(50).
    u = np.array([[0.75, 0.0, 0.0, 2.0, -0.6],
                  [0.0, 12 / 5, 0.0, 3.0, 0.0],
                  [0.0, 0.0, 0.0, 6.0, 0.8]])
    w = np.array([2.0, 0.5, 7.0, 1.0, 3.0])
    m = 1836.0
    sp = _Sp(1.0, m, np.zeros((3, 5)), u, w)
    gm1 = np.array([0.25, 1.6, 0.0, math.sqrt(50.0) - 1.0, math.sqrt(2.0) - 1.0])
    expect = float(np.sum(w * m * gm1))
    assert abs(oracle.kinetic_energy(sp) - expect) < 1e-14 * expect


def test_kinetic_energy_small_momentum_series():
    # gamma - 1 = u^2/2 - u^4/8 + u^6/16 - ...: the value must keep its
    # relative accuracy at |u| << 1 (no cancellation in sqrt(1 + u^2) - 1).
    for a in (1e-3, 1e-5, 1e-7):
        u = np.array([[a], [0.0], [0.0]])
        sp = _Sp(-1.0, 1.0, np.zeros((3, 1)), u, np.array([1.0]))
        u2 = a * a
        series = u2 / 2 - u2 * u2 / 8 + u2 ** 3 / 16
        assert abs(oracle.kinetic_energy(sp) - series) < 1e-15 * series
