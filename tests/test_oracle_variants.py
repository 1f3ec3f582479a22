"""Pins of the oracle's pusher and gather variants.

Vay pusher: a pure electric field is a plain kick; a pure magnetic field
keeps gamma; a particle moving at a relativistic E x B drift velocity feels
E + v x B = 0 and keeps its momentum exactly (Boris's average does not).
Galerkin gather: uniform fields are reproduced; along an axis where a
component sits at half-integer points the shape is one order lower, so a
quadratic profile along it is interpolated with the lower order's closed
form (nearest node for order 1, linear interpolation for order 2), while
along its other axes the full order applies (a quadratic reproduced as
x^2 + 1/4 by the order-2 B-spline).
"""
import math

import numpy as np
import pytest

import oracle


def test_vay_pure_electric_kick():
    u = np.array([0.3, -0.2, 0.9])
    E = np.array([0.01, 0.02, -0.03])
    out = oracle.vay(-1.0, 1.0, 0.5, E, np.zeros(3), u)
    np.testing.assert_allclose(out, u + (-1.0 / 1.0) * 0.5 * E, atol=1e-16)


def test_vay_pure_magnetic_keeps_gamma():
    rng = np.random.default_rng(4)
    for _ in range(20):
        u = rng.normal(size=3) * 3
        B = rng.normal(size=3)
        out = u.copy()
        for _ in range(50):
            out = oracle.vay(1.0, 1.0, 0.7, np.zeros(3), B, out)
        assert abs(np.linalg.norm(out) - np.linalg.norm(u)) < 1e-12 * np.linalg.norm(u)


def test_vay_relativistic_exb_drift_is_exact_where_boris_is_not():
    B0 = 1.5
    vd = 0.9
    B = np.array([0.0, 0.0, B0])
    E = np.array([-vd * B0, 0.0, 0.0])        # E = -v_d x B, v_d along y
    gd = 1.0 / math.sqrt(1.0 - vd * vd)
    u0 = np.array([0.0, gd * vd, 0.0])
    uv, ub = u0.copy(), u0.copy()
    for _ in range(1000):
        uv = oracle.vay(-1.0, 1.0, 0.3, E, B, uv)
        ub = oracle.boris(-1.0, 1.0, 0.3, E, B, ub)
    assert np.max(np.abs(uv - u0)) < 1e-12
    assert np.max(np.abs(ub - u0)) > 1e-3


def _grid(order, n=(12, 10, 11)):
    return oracle.make_grid(3, n, (1.0, 1.0, 1.0), 0.3, order)


@pytest.mark.parametrize("order", (1, 2, 3))
def test_galerkin_uniform_fields(order):
    g = _grid(order)
    N = 12 * 10 * 11
    vals = [0.3, -0.2, 0.5, 0.7, -0.1, 0.4]
    E = np.array([np.full(N, v) for v in vals[:3]])
    B = np.array([np.full(N, v) for v in vals[3:]])
    for xi in ([5.3, 4.7, 6.1], [2.5, 3.5, 4.5], [7.0, 1.25, 9.9]):
        Ep, Bp = oracle.gather_galerkin(g, E, B, np.array(xi))
        np.testing.assert_allclose(Ep, vals[:3], atol=1e-15)
        np.testing.assert_allclose(Bp, vals[3:], atol=1e-15)


def test_galerkin_lower_order_on_the_staggered_axis():
    # E_x at (i + 1/2, j, k) = (i + 1/2 - c)^2: staggered along x only.
    n = (16, 10, 10)
    N = 1600
    c = 8.0
    i = np.arange(n[0])
    ex = np.broadcast_to(((i + 0.5 - c) ** 2)[None, None, :], (n[2], n[1], n[0])).ravel()
    E = np.zeros((3, N))
    B = np.zeros((3, N))
    E[0] = ex
    for x in (7.3, 8.0, 8.9):
        # order 1 -> order 0 along x: the nearest E_x node
        Ep, _ = oracle.gather_galerkin(_grid(1, n), E, B, np.array([x, 4.2, 5.6]))
        node = math.floor(x - 0.5 + 0.5) + 0.5
        assert abs(Ep[0] - (node - c) ** 2) < 1e-13
        # order 2 -> order 1 along x: linear interpolation of the quadratic
        Ep, _ = oracle.gather_galerkin(_grid(2, n), E, B, np.array([x, 4.2, 5.6]))
        lo = math.floor(x - 0.5) + 0.5
        a = x - lo
        lin = (1 - a) * (lo - c) ** 2 + a * (lo + 1 - c) ** 2
        assert abs(Ep[0] - lin) < 1e-13
        # the default gather keeps order 2: x^2 + 1/4 for the B-spline
        Ep, _ = oracle.gather(_grid(2, n), E, B, np.array([x, 4.2, 5.6]))
        assert abs(Ep[0] - ((x - c) ** 2 + 0.25)) < 1e-13


def test_galerkin_full_order_across():
    # E_x varying quadratically along z (not staggered there): the full
    # order-2 B-spline, giving (z - c)^2 + 1/4
    n = (10, 10, 16)
    N = 1600
    c = 8.0
    k = np.arange(n[2])
    ex = np.broadcast_to(((k - c) ** 2)[:, None, None], (n[2], n[1], n[0])).ravel()
    E = np.zeros((3, N))
    E[0] = ex
    for z in (7.3, 8.0, 8.6):
        Ep, _ = oracle.gather_galerkin(_grid(2, n), E, np.zeros_like(E), np.array([4.4, 5.5, z]))
        assert abs(Ep[0] - ((z - c) ** 2 + 0.25)) < 1e-13
