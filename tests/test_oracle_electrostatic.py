"""Pins of the oracle's electrostatic variant.

Poisson: div E = rho - <rho> with the Yee differences holds to rounding for
any charge (Gauss's law); a single Fourier mode of rho gives phi = rho /
lambda_m with lambda_m = (2 - 2 cos(2 pi m / n)) / dx^2 exactly.
Particle update: in a field set directly, u changes by q E dt / m and x
advances with the new u.  Whole steps: a cold electron plasma displaced by
a long sinusoid oscillates at the plasma frequency (leapfrog-corrected).
"""
import math

import numpy as np
import pytest

import oracle
import pic_inputs as pi


@pytest.mark.parametrize("dim,order", ((3, 1), (3, 3), (2, 2)))
def test_gauss_law_holds(dim, order):
    wl = pi.uniform_box((10, 8, 12), 3, 0.05, 0.1, order, 9400 + dim, "cpu", tile=(4, 4, 4),
                        dim=dim)
    box = wl.boxes[0]
    g = oracle.make_grid(dim, box.n, (1.0, 1.3, 0.8) if dim == 3 else (1.0, 1.0, 0.8),
                         box.dt, order)
    sps = [p.numpy() for p in wl.species]
    r = oracle.rho(g, sps, box.ncells)
    phi = oracle.poisson_periodic(g, r)
    E = oracle.es_field(g, phi)
    div = oracle.div_j(g, E, box.ncells)
    assert np.max(np.abs(div - (r - r.mean()))) < 1e-12 * np.max(np.abs(r - r.mean()))
    assert abs(np.mean(phi)) < 1e-14


@pytest.mark.parametrize("m", (1, 3))
def test_single_mode(m):
    n = (16, 4, 6)
    dx = 0.75
    g = oracle.make_grid(3, n, (dx, 1.0, 1.0), 0.3, 1)
    i = np.arange(n[0])
    prof = np.cos(2 * math.pi * m * i / n[0])
    rho = np.broadcast_to(prof[None, None, :], (n[2], n[1], n[0])).ravel().copy()
    lam = (2.0 - 2.0 * math.cos(2 * math.pi * m / n[0])) / dx ** 2
    phi = oracle.poisson_periodic(g, rho)
    np.testing.assert_allclose(phi, rho / lam, atol=1e-14)
    E = oracle.es_field(g, phi)
    ex = -(np.cos(2 * math.pi * m * (i + 1) / n[0]) - prof) / (lam * dx)
    np.testing.assert_allclose(E[0], np.broadcast_to(ex[None, None, :], (n[2], n[1], n[0])).ravel(),
                               atol=1e-14)
    assert np.all(E[1] == 0.0) and np.all(np.abs(E[2]) < 1e-15)


def test_kick_in_a_given_field():
    n = (6, 6, 6)
    g = oracle.make_grid(3, n, (1.0, 1.0, 1.0), pi.DT3, 2)
    N = 216
    E = np.zeros((3, N))
    E[0][:] = 0.02
    E[2][:] = -0.01

    class S:
        pass

    s = S()
    s.q, s.m = -1.0, 1.0
    s.x = np.array([[2.3], [1.1], [4.9]])
    s.u = np.array([[0.1], [0.0], [-0.2]])
    s.w = np.array([1.0])
    x0, u0 = s.x.copy(), s.u.copy()
    oracle.es_particles_step(g, E, [s])
    du = s.u[:, 0] - u0[:, 0]
    np.testing.assert_allclose(du, [-0.02 * g.dt, 0.0, 0.01 * g.dt], atol=1e-16)
    gam = math.sqrt(1.0 + s.u[:, 0] @ s.u[:, 0])
    np.testing.assert_allclose(s.x[:, 0], x0[:, 0] + g.dt * s.u[:, 0] / gam, atol=1e-14)


def test_cold_plasma_oscillates_at_the_plasma_frequency():
    n = (2, 2, 64)
    n0 = 0.01
    ppc = 4
    box = pi.Box(3, n, pi.DT3, 1)
    g = oracle.make_grid(3, n, (1.0, 1.0, 1.0), box.dt, 1)
    nc = n[0] * n[1] * n[2]
    cells = np.repeat(np.arange(nc), ppc)
    sub = (np.arange(cells.size) % ppc + 0.5) / ppc
    x = np.stack([cells % n[0] + 0.5, (cells // n[0]) % n[1] + 0.5, cells // (n[0] * n[1]) + sub])
    k = 2 * math.pi / n[2]
    x[2] = np.mod(x[2] + 0.05 * np.sin(k * x[2]), n[2])

    class S:
        pass

    s = S()
    s.q, s.m = -1.0, 1.0
    s.x = np.ascontiguousarray(x)
    s.u = np.zeros_like(s.x)
    s.w = np.full(cells.size, n0 / ppc)
    amp = []
    steps = 260
    for _ in range(steps):
        _, _, E = oracle.es_step(g, [s], nc)
        ez = E[2].reshape(n[2], n[1], n[0])[:, 0, 0]
        amp.append(np.sum(ez * np.sin(k * (np.arange(n[2]) + 0.5))))
    a = np.array(amp)
    zc = np.nonzero(np.sign(a[1:]) != np.sign(a[:-1]))[0]
    # crossings are half a period apart
    period_steps = 2.0 * (zc[-1] - zc[0]) / (len(zc) - 1)
    wp = math.sqrt(n0)
    w_leapfrog = 2.0 / g.dt * math.asin(wp * g.dt / 2.0)
    w = 2 * math.pi / (period_steps * g.dt)
    assert len(zc) >= 4
    assert abs(w / w_leapfrog - 1.0) < 0.02, (w, w_leapfrog)
