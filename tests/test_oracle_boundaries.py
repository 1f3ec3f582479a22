"""Pins of the oracle's laser-plasma boundaries against closed forms.

Absorbing layers: with no layer the step is the plain Yee step, bit for bit;
E_z and B_z uniform across x and y have no curl, so each decays by exactly
exp(-sigma dt) per step with sigma taken at its own Yee point; a plane
pulse at normal incidence is absorbed (almost nothing comes back), while
the same pulse without layers keeps its energy.

Antenna: in a box uniform across x and y the sheet radiates plane waves of
amplitude E0 to both sides (continuum: E = -K / 2), symmetric about the
sheet, travelling at c.

Moving window: a vacuum laser pulse moving at c stays put in a frame that
shifts one cell every 1/dt steps; a shift moves particles one cell back and
drops those that leave.
"""
import math

import numpy as np
import pytest

import oracle
import pic_inputs as pi


def _plane_box(nz, dt=None, n=(2, 2)):
    dt = dt if dt is not None else pi.DT3
    return oracle.make_grid(3, (n[0], n[1], nz), (1.0, 1.0, 1.0), dt, 1)


def test_no_layer_is_plain_yee():
    box = pi.Box(3, (6, 5, 12), pi.DT3, 1)
    E, B = pi.fourier_fields(box, 3, 0.1, 9001, "cpu")
    g = oracle.make_grid(3, box.n, box.dx, box.dt, 1)
    E1, B1 = E.numpy().copy(), B.numpy().copy()
    E2, B2 = E.numpy().copy(), B.numpy().copy()
    J = np.random.default_rng(3).normal(size=E1.shape) * 1e-3
    oracle.fdtd_step(g, E1, B1, J)
    oracle.fdtd_step_absorb(g, E2, B2, J, oracle.absorber(0, 5.0, 3))
    np.testing.assert_array_equal(E1, E2)
    np.testing.assert_array_equal(B1, B2)


@pytest.mark.parametrize("zoff", (0.0, 5.0))
def test_uniform_axial_fields_decay_exactly(zoff):
    # E_z and B_z uniform across x, y (any profile along z) have no curl, so
    # each decays by exactly exp(-sigma dt) per step, sigma at its own Yee
    # point: E_z at k + 1/2, B_z at k; the other components stay zero.
    nz = 20
    g = _plane_box(nz, n=(3, 4))
    a = oracle.absorber(6, 1.5, 2)
    N = 3 * 4 * nz
    ez0, bz0 = 0.3, -0.7
    E = np.zeros((3, N))
    B = np.zeros((3, N))
    E[2][:] = ez0
    B[2][:] = bz0
    J = np.zeros_like(E)
    steps = 7
    for _ in range(steps):
        oracle.fdtd_step_absorb(g, E, B, J, a, zoff)
    k = np.repeat(np.arange(nz), 12).astype(np.float64)
    for F, off, v in ((E[2], 0.5, ez0), (B[2], 0.0, bz0)):
        z = np.mod(k + off - zoff, nz)
        sig = np.array([oracle.absorber_sigma(a, zz, nz) for zz in z])
        np.testing.assert_allclose(F, v * np.exp(-sig * g.dt * steps), rtol=1e-13, atol=1e-16)
    for F in (E[0], E[1], B[0], B[1]):
        assert np.all(F == 0.0)


def _pulse(g, nz, z0, L):
    """A +z plane pulse Ex = By (Gaussian envelope, lambda = 20 cells) at
    each component's own Yee points; B half a step behind is ignored (the
    small backward part it leaves is part of the measured budget)."""
    N = g.n[0] * g.n[1] * nz
    k = np.repeat(np.arange(nz), g.n[0] * g.n[1]).astype(np.float64)
    f = lambda z: np.exp(-((z - z0) / L) ** 2) * np.sin(2 * math.pi * z / 20.0)
    E = np.zeros((3, N))
    B = np.zeros((3, N))
    E[0] = f(k)
    B[1] = f(k + 0.5)
    return E, B


def test_pulse_is_absorbed_at_normal_incidence():
    nz = 240
    g = _plane_box(nz)
    E, B = _pulse(g, nz, 150.0, 12.0)
    J = np.zeros_like(E)
    w0 = oracle.field_energy(g, E, B)
    a = oracle.absorber(24, 4.0, 3)
    # the pulse travels +z, enters the top layer, and anything it reflects
    # or sends around the (periodic) box ends up in the interior
    for _ in range(int(200 / g.dt)):
        oracle.fdtd_step_absorb(g, E, B, J, a)
    inner = slice(24 * 4, (nz - 24) * 4)
    w_in = 0.5 * (np.sum(E[:, inner] ** 2) + np.sum(B[:, inner] ** 2))
    assert w_in < 1e-5 * w0, w_in / w0
    # without layers the energy stays (plain Yee keeps it to its leapfrog
    # oscillation)
    E2, B2 = _pulse(g, nz, 150.0, 12.0)
    for _ in range(int(200 / g.dt)):
        oracle.fdtd_step_absorb(g, E2, B2, J, oracle.absorber(0, 0.0, 3))
    assert oracle.field_energy(g, E2, B2) > 0.98 * w0


def test_antenna_emits_amplitude_e0_both_ways():
    nz = 400
    g = _plane_box(nz)
    E = np.zeros((3, 4 * nz))
    B = np.zeros_like(E)
    J = np.zeros_like(E)
    a = oracle.absorber(30, 3.0, 3)
    omega = 2 * math.pi / 20.0
    ka = 200
    an = oracle.antenna(ka, 0.7, omega, 1e6, 1.0, 1.0, 60.0, 1e9)   # plane, steady wave
    steps = int(150 / g.dt)
    for n in range(steps):
        J[:] = 0.0
        oracle.antenna_add(g, J, an, (n + 0.5) * g.dt)
        oracle.fdtd_step_absorb(g, E, B, J, a)
    ex = E[0].reshape(nz, 4)[:, 0]
    up = ex[ka + 20: ka + 100]
    down = ex[ka - 100: ka - 20]
    assert abs(np.max(np.abs(up)) / 0.7 - 1.0) < 0.02
    assert abs(np.max(np.abs(down)) / 0.7 - 1.0) < 0.02
    # symmetric about the sheet: E_x(z_a + d) = E_x(z_a - d) (both travel away)
    d = np.arange(10, 90)
    np.testing.assert_allclose(ex[ka + d], ex[ka - d], atol=0.02 * 0.7)


def test_window_keeps_a_vacuum_pulse_in_place():
    nz = 160
    g = _plane_box(nz)
    E, B = _pulse(g, nz, 80.0, 10.0)
    J = np.zeros_like(E)
    a = oracle.absorber(16, 3.0, 3)
    k = np.repeat(np.arange(nz), 4).astype(np.float64)

    def centroid():
        w = E[0] ** 2 + E[1] ** 2 + E[2] ** 2
        return float(np.sum(w * k) / np.sum(w))

    c0 = centroid()
    travelled, shifts = 0.0, 0
    for _ in range(int(40 / g.dt)):
        oracle.fdtd_step_absorb(g, E, B, J, a)
        travelled += g.dt
        while travelled - shifts >= 1.0:
            oracle.window_shift_fields(g, E, B)
            shifts += 1
    assert shifts == 40 or shifts == 39
    assert abs(centroid() - c0) < 1.0


def test_window_shift_particles():
    g = oracle.make_grid(3, (4, 4, 10), (1.0, 1.0, 1.0), pi.DT3, 2)
    rng = np.random.default_rng(8)
    n = 50
    x = np.stack([rng.uniform(0, 4, n), rng.uniform(0, 4, n), rng.uniform(0, 10, n)])
    u = rng.normal(size=(3, n))
    w = rng.uniform(size=n)

    class S:
        pass

    sp = S()
    sp.q, sp.m = -1.0, 1.0
    sp.x, sp.u, sp.w = x.copy(), u.copy(), w.copy()
    m = oracle.window_shift_particles(g, sp)
    keep = x[2] >= 1.0
    assert m == int(np.sum(keep))
    np.testing.assert_array_equal(sp.x[:2, :m], x[:2, keep])
    np.testing.assert_array_equal(sp.x[2, :m], x[2, keep] - 1.0)
    np.testing.assert_array_equal(sp.u[:, :m], u[:, keep])
    np.testing.assert_array_equal(sp.w[:m], w[keep])
