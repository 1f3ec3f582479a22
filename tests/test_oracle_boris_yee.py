"""Pins of the oracle's Boris push and Yee solver against closed forms.

Boris: in a pure magnetic field the step is an exact rotation of u by
2 atan(|q| B dt / (2 m gamma)) with |u| conserved; with crossed uniform
E and B (|E| < |B|) the discrete E x B drift has an exact fixed point,
derived by requiring u_new == u in the scheme's own equations; a pure
electric field is a plain kick q E dt / m.

Yee: a discrete plane wave of the staggered leapfrog keeps its amplitude
and advances its phase by omega dt per step where sin^2(omega dt/2)/dt^2
equals the sum over axes of sin^2(k_d dx_d/2)/dx_d^2; div B is preserved;
the leapfrog energy 1/2 (E^n.E^n + B^(n-1/2).B^(n+1/2)) is invariant.
"""
import math

import numpy as np
import pytest

import oracle


def test_boris_gyration_angle_and_norm():
    rng = np.random.default_rng(11)
    for _ in range(50):
        q = rng.choice([-1.0, 1.0])
        m = rng.choice([1.0, 1836.0])
        dt = rng.uniform(0.1, 1.0)
        Bz = rng.uniform(0.1, 3.0) * m
        u = np.array([rng.normal(), rng.normal(), rng.normal()])
        un = oracle.boris(q, m, dt, np.zeros(3), np.array([0.0, 0.0, Bz]), u)
        gam = math.sqrt(1 + u @ u)
        assert abs(np.linalg.norm(un) - np.linalg.norm(u)) < 1e-14 * np.linalg.norm(u) + 1e-15
        assert un[2] == u[2]
        ang = math.atan2(u[0] * un[1] - u[1] * un[0], u[0] * un[0] + u[1] * un[1])
        expect = -math.copysign(2.0 * math.atan(abs(q) * Bz * dt / (2 * m * gam)), q)
        assert abs(ang - expect) < 1e-13


def test_boris_exb_discrete_fixed_point():
    # E along x, B along z: drift along -y.  The fixed point solves
    # h E = (h B / gamma_minus) U with gamma_minus = sqrt(1 + h^2 E^2 + U^2).
    for q in (-1.0, 1.0):
        for (E, B, dt, m) in ((0.3, 1.0, 0.5, 1.0), (0.05, 0.2, 0.9, 1.0), (0.9, 1.0, 0.1, 3.0)):
            h = q * dt / (2 * m)
            U = (E / B) * math.sqrt((1 + h * h * E * E) / (1 - E * E / (B * B)))
            u = np.array([0.0, -U, 0.0])
            un = u.copy()
            for _ in range(1000):
                un = oracle.boris(q, m, dt, np.array([E, 0, 0]), np.array([0, 0, B]), un)
            assert np.max(np.abs(un - u)) < 1e-12
            # and the drift velocity tends to E x B / B^2 as dt -> 0
            v = U / math.sqrt(1 + U * U)
            if dt <= 0.1:
                h0 = 0.0
                U0 = (E / B) / math.sqrt(1 - E * E / (B * B))
                assert abs(v - U0 / math.sqrt(1 + U0 * U0)) < 1e-2


def test_boris_pure_electric_kick():
    rng = np.random.default_rng(12)
    for _ in range(20):
        q, m, dt = rng.choice([-1.0, 1.0]), rng.uniform(0.5, 3), rng.uniform(0.1, 1)
        E = rng.standard_normal(3)
        u = rng.standard_normal(3)
        un = oracle.boris(q, m, dt, E, np.zeros(3), u)
        assert np.allclose(un, u + q * dt / m * E, rtol=0, atol=1e-14)


# ------------------------------------------------------------------ Yee

def _khat(k, dx):
    return 2.0 * math.sin(k * dx / 2.0) / dx


def _omega(kvec, dx, dt):
    s = sum(_khat(k, d) ** 2 for k, d in zip(kvec, dx))
    return 2.0 / dt * math.asin(dt * math.sqrt(s) / 2.0)


def _grid_idx(n):
    i, j, k = np.meshgrid(np.arange(n[0]), np.arange(n[1]), np.arange(n[2]), indexing="ij")
    f = lambda a: a.transpose(2, 1, 0).reshape(-1).astype(np.float64)
    return f(i), f(j), f(k)


@pytest.mark.parametrize("dim,plane,dx", [(3, "xy", (1.0, 1.0, 1.0)), (3, "xz", (1.0, 1.3, 0.8)),
                                          (2, "xz", (1.0, 1.0, 1.0)), (3, "yz", (0.9, 1.1, 1.0))])
def test_yee_plane_wave_dispersion(dim, plane, dx):
    n = (16, 12, 10) if dim == 3 else (16, 1, 10)
    cfl = 1.0 / math.sqrt(sum(1.0 / d ** 2 for d in (dx if dim == 3 else (dx[0], dx[2]))))
    dt = 0.9 * cfl
    g = oracle.make_grid(dim, n, dx, dt, 1)
    I, Jj, K = _grid_idx(n)
    N = n[0] * n[1] * n[2]
    # TM-like mode in the given plane: E along the normal axis c, B in-plane.
    a, b = {"xy": (0, 1), "xz": (0, 2), "yz": (1, 2)}[plane]
    c = 3 - a - b
    kv = [0.0, 0.0, 0.0]
    kv[a] = 2 * math.pi * 2 / (n[a] * dx[a])
    kv[b] = 2 * math.pi * 1 / (n[b] * dx[b])
    om = _omega(kv, dx, dt)
    Om = 2 * math.sin(om * dt / 2) / dt
    idx = [I, Jj, K]

    def phase(shift, t):
        # shift: per-axis half-cell offsets of the component's Yee point
        return sum(kv[d] * (idx[d] + shift[d]) * dx[d] for d in range(3)) - om * t

    def sh(comp, kind):
        return [0.5 if ((d == comp) if kind == "E" else (d != comp)) and not (dim == 2 and d == 1)
                else 0.0 for d in range(3)]

    E = np.zeros((3, N)); B = np.zeros((3, N)); J = np.zeros((3, N))
    E[c] = np.cos(phase(sh(c, "E"), 0.0))
    # Faraday on the mode: (curl E)_comp = eps(comp, other, c) d_other E_c
    # and the discrete d_other of cos(theta) is -khat sin(theta at the B
    # point); B(n+1/2) - B(n-1/2) = A Om dt sin(...) then gives
    # A = eps khat / Om, and B at integer times is A cos(om dt/2) cos(...).
    eps = {(0, 1, 2): 1, (1, 2, 0): 1, (2, 0, 1): 1, (0, 2, 1): -1, (2, 1, 0): -1, (1, 0, 2): -1}
    for comp in (a, b):
        other = b if comp == a else a
        # (curl E)_comp = eps(comp, other, c) d_other E_c
        coef = eps[(comp, other, c)] * _khat(kv[other], dx[other]) / Om
        B[comp] = coef * math.cos(om * dt / 2) * np.cos(phase(sh(comp, "B"), 0.0))
    steps = 40
    for _ in range(steps):
        oracle.fdtd_step(g, E, B, J)
    ref = np.cos(phase(sh(c, "E"), steps * dt))
    assert np.max(np.abs(E[c] - ref)) < 1e-11
    for comp in (a, b):
        other = b if comp == a else a
        coef = eps[(comp, other, c)] * _khat(kv[other], dx[other]) / Om
        refB = coef * math.cos(om * dt / 2) * np.cos(phase(sh(comp, "B"), steps * dt))
        assert np.max(np.abs(B[comp] - refB)) < 1e-11


def _div_b(n, B, dx):
    """Discrete divergence at cell centres (i+1/2, j+1/2, k+1/2)."""
    r = lambda F: F.reshape(n[2], n[1], n[0])
    bx, by, bz = r(B[0]), r(B[1]), r(B[2])
    return ((np.roll(bx, -1, 2) - bx) / dx[0] + (np.roll(by, -1, 1) - by) / dx[1] +
            (np.roll(bz, -1, 0) - bz) / dx[2])


def test_yee_div_b_and_energy_invariants():
    n = (8, 7, 6)
    dx = (1.0, 1.0, 1.0)
    dt = 0.95 / math.sqrt(3)
    g = oracle.make_grid(3, n, dx, dt, 1)
    N = n[0] * n[1] * n[2]
    rng = np.random.default_rng(13)
    E = rng.standard_normal((3, N)); B = rng.standard_normal((3, N)); J = np.zeros((3, N))
    d0 = _div_b(n, B, dx)

    def leapfrog_energy(E, B):
        Bm, Bp = B.copy(), B.copy()
        oracle.faraday(g, E, Bm, -0.5 * dt)     # B^(n-1/2)
        oracle.faraday(g, E, Bp, 0.5 * dt)      # B^(n+1/2)
        return 0.5 * (np.sum(E * E) + np.sum(Bm * Bp))

    e0 = leapfrog_energy(E, B)
    for _ in range(25):
        oracle.fdtd_step(g, E, B, J)
    assert np.max(np.abs(_div_b(n, B, dx) - d0)) < 1e-12
    assert abs(leapfrog_energy(E, B) - e0) < 1e-11 * abs(e0)


def test_yee_2d_equals_3d_with_one_y_cell():
    n = (9, 1, 7)
    rng = np.random.default_rng(14)
    E = rng.standard_normal((3, 63)); B = rng.standard_normal((3, 63)); J = rng.standard_normal((3, 63))
    E2, B2 = E.copy(), B.copy()
    g3 = oracle.make_grid(3, n, (1, 1, 1), 0.6, 1)
    g2 = oracle.make_grid(2, n, (1, 1, 1), 0.6, 1)
    for _ in range(5):
        oracle.fdtd_step(g3, E, B, J)
        oracle.fdtd_step(g2, E2, B2, J)
    assert np.array_equal(E, E2) and np.array_equal(B, B2)
