"""Pins of the oracle's Ampere update and of its particle step with the
pusher / gather options, against results fixed without the oracle's own
arithmetic:

* Ampere with B = 0: E changes by exactly -dt J at every E point;
* Ampere with a single B_z mode along x: E_y changes by dt times the
  one-cell difference -(B_z(i+1/2) - B_z(i-1/2)) / dx, a closed form;
* the option step with the default pusher and gather is the default step,
  bit for bit;
* with B = 0 the Vay pusher is a plain electric kick, so it reproduces the
  Boris step;
* the Galerkin gather of uniform fields is the uniform value, so the
  option step reproduces the default step;
* a particle at the relativistic E x B drift velocity keeps its momentum
  exactly through whole Vay steps and advances by dt v per step.
"""
import math

import numpy as np
import pytest

import oracle


class _Sp:
    def __init__(self, q, m, x, u, w):
        self.q, self.m = q, m
        self.x = np.array(x, dtype=np.float64, order="C", copy=True)
        self.u = np.array(u, dtype=np.float64, order="C", copy=True)
        self.w = np.array(w, dtype=np.float64, order="C", copy=True)


def _plasma(n, npart, seed, u_scale=0.3):
    rng = np.random.default_rng(seed)
    x = rng.uniform(0.0, 1.0, size=(3, npart)) * np.array(n, dtype=np.float64)[:, None]
    u = rng.normal(size=(3, npart)) * u_scale
    w = rng.uniform(0.5, 1.5, size=npart)
    return x, u, w


def test_ampere_with_zero_b_is_minus_dt_j():
    n = (6, 5, 7)
    g = oracle.make_grid(3, n, (1.0, 1.0, 1.0), 0.4, 1)
    N = 6 * 5 * 7
    rng = np.random.default_rng(1)
    E0 = rng.normal(size=(3, N))
    J = rng.normal(size=(3, N))
    E = E0.copy()
    oracle.ampere(g, E, np.zeros((3, N)), J, 0.4)
    np.testing.assert_allclose(E, E0 - 0.4 * J, rtol=0, atol=1e-15)


def test_ampere_single_bz_mode():
    n = (16, 4, 4)
    dx = 0.7
    dt = 0.3
    g = oracle.make_grid(3, n, (dx, 1.0, 1.0), dt, 1)
    N = 16 * 4 * 4
    k = 2 * math.pi * 3 / (n[0] * dx)
    i = np.arange(n[0])
    bz_row = np.sin(k * (i + 0.5) * dx)          # B_z at x = (i + 1/2) dx
    B = np.zeros((3, N))
    B[2] = np.broadcast_to(bz_row[None, None, :], (4, 4, 16)).ravel()
    E = np.zeros((3, N))
    oracle.ampere(g, E, B, np.zeros((3, N)), dt)
    # (curl B)_y = -dBz/dx at E_y's point (i, j + 1/2, k)
    dbz = (bz_row - np.roll(bz_row, 1)) / dx
    ey = np.broadcast_to((-dt * dbz)[None, None, :], (4, 4, 16)).ravel()
    np.testing.assert_allclose(E[1], ey, rtol=0, atol=1e-14)
    assert np.max(np.abs(E[0])) == 0.0 and np.max(np.abs(E[2])) == 0.0


def _fields(N, seed, uniform=False):
    rng = np.random.default_rng(seed)
    if uniform:
        E = np.repeat(rng.normal(size=(3, 1)) * 0.05, N, axis=1)
        B = np.repeat(rng.normal(size=(3, 1)) * 0.05, N, axis=1)
    else:
        E = rng.normal(size=(3, N)) * 0.05
        B = rng.normal(size=(3, N)) * 0.05
    return E, B


@pytest.mark.parametrize("order", (1, 2, 3))
def test_default_options_are_the_default_step(order):
    n = (8, 7, 9)
    g = oracle.make_grid(3, n, (1.0, 1.0, 1.0), 0.5, order)
    N = 8 * 7 * 9
    E, B = _fields(N, 5)
    x, u, w = _plasma(n, 300, 6)
    a, b = _Sp(-1.0, 1.0, x, u, w), _Sp(-1.0, 1.0, x, u, w)
    Ja, Jb = np.zeros((3, N)), np.zeros((3, N))
    oracle.particles_step(g, E.copy(), B.copy(), Ja, [a])
    oracle.particles_step_opts(g, E.copy(), B.copy(), Jb, [b], 0, 0)
    assert np.array_equal(Ja, Jb) and np.array_equal(a.x, b.x) and np.array_equal(a.u, b.u)


@pytest.mark.parametrize("order", (1, 3))
def test_vay_without_b_is_the_boris_step(order):
    n = (8, 7, 9)
    g = oracle.make_grid(3, n, (1.0, 1.0, 1.0), 0.5, order)
    N = 8 * 7 * 9
    E, _ = _fields(N, 7)
    B = np.zeros((3, N))
    x, u, w = _plasma(n, 300, 8)
    a, b = _Sp(1.0, 3.0, x, u, w), _Sp(1.0, 3.0, x, u, w)
    Ja, Jb = np.zeros((3, N)), np.zeros((3, N))
    oracle.particles_step(g, E.copy(), B.copy(), Ja, [a])
    oracle.particles_step_opts(g, E.copy(), B.copy(), Jb, [b], 1, 0)
    np.testing.assert_allclose(b.u, a.u, rtol=1e-14, atol=1e-16)
    np.testing.assert_allclose(b.x, a.x, rtol=0, atol=1e-12)
    np.testing.assert_allclose(Jb, Ja, rtol=0, atol=1e-12 * np.max(np.abs(Ja)))


@pytest.mark.parametrize("order", (1, 2, 3))
def test_galerkin_step_in_uniform_fields_is_the_default_step(order):
    n = (8, 7, 9)
    g = oracle.make_grid(3, n, (1.0, 1.0, 1.0), 0.5, order)
    N = 8 * 7 * 9
    E, B = _fields(N, 9, uniform=True)
    x, u, w = _plasma(n, 300, 10)
    a, b = _Sp(-1.0, 1.0, x, u, w), _Sp(-1.0, 1.0, x, u, w)
    Ja, Jb = np.zeros((3, N)), np.zeros((3, N))
    oracle.particles_step(g, E.copy(), B.copy(), Ja, [a])
    oracle.particles_step_opts(g, E.copy(), B.copy(), Jb, [b], 0, 1)
    np.testing.assert_allclose(b.u, a.u, rtol=1e-14, atol=1e-16)
    np.testing.assert_allclose(b.x, a.x, rtol=0, atol=1e-12)
    np.testing.assert_allclose(Jb, Ja, rtol=0, atol=1e-12 * np.max(np.abs(Ja)))


def test_vay_steps_keep_the_relativistic_drift():
    n = (16, 16, 16)
    dt = 0.5
    g = oracle.make_grid(3, n, (1.0, 1.0, 1.0), dt, 2)
    N = 16 ** 3
    B0, vd = 1.2, 0.8
    E = np.zeros((3, N))
    B = np.zeros((3, N))
    B[2] = B0
    E[0] = -vd * B0                  # E = -v_d x B with v_d along y
    gd = 1.0 / math.sqrt(1.0 - vd * vd)
    sp = _Sp(-1.0, 1.0, [[5.25], [3.5], [7.75]], [[0.0], [gd * vd], [0.0]], [1.0])
    y0 = sp.x[1, 0]
    for k in range(1, 9):
        J = np.zeros((3, N))
        oracle.particles_step_opts(g, E.copy(), B.copy(), J, [sp], 1, 0)
        assert abs(sp.u[0, 0]) < 1e-13 and abs(sp.u[2, 0]) < 1e-13
        assert abs(sp.u[1, 0] - gd * vd) < 1e-13
        assert abs(sp.x[0, 0] - 5.25) < 1e-12 and abs(sp.x[2, 0] - 7.75) < 1e-12
        assert abs(sp.x[1, 0] - (y0 + k * dt * vd) % 16) < 1e-12
