"""Pins of the oracle's B-spline shape factors and field gather.

Shapes: the order-n B-spline is the unit box convolved with the order n-1
spline (checked by quadrature, starting from the box itself), has unit sum
over integer translates, reproduces linear functions and has, for
orders >= 2, sampled variance (n+1)/12 (and zero third moment at order 3).  Gather: brute-force sums over every grid point, exact
reproduction of uniform and linear fields at each component's own Yee
stagger, and the 2D path equal to the 3D path with one cell along y.
"""
import math

import numpy as np
import pytest
from scipy.integrate import quad

import oracle

ORDERS = (1, 2, 3)


def S(o, a):
    return oracle.shape(o, a)


def box(a):
    return 1.0 if abs(a) < 0.5 else (0.5 if abs(a) == 0.5 else 0.0)


@pytest.mark.parametrize("o", ORDERS)
def test_shape_is_box_convolution(o):
    lower = box if o == 1 else (lambda t: S(o - 1, t))
    rng = np.random.default_rng(1)
    for a in list(rng.uniform(-2.6, 2.6, 40)) + [0.0, 0.5, 1.0, 1.5, 2.0]:
        pts = [p for p in np.arange(-3.0, 3.01, 0.5) if a - 0.5 < p < a + 0.5]
        ref, _ = quad(lower, a - 0.5, a + 0.5, points=pts or None, epsabs=1e-14, epsrel=1e-14)
        assert abs(S(o, a) - ref) < 1e-12, (o, a)


@pytest.mark.parametrize("o", ORDERS)
def test_shape_moments(o):
    rng = np.random.default_rng(2)
    for xi in rng.uniform(-5, 5, 200):
        nodes = np.arange(math.floor(xi) - 3, math.floor(xi) + 5)
        s = np.array([S(o, xi - i) for i in nodes])
        assert abs(s.sum() - 1.0) < 4e-16
        assert abs((nodes * s).sum() - xi) < 4e-15
        # Sampled moments of degree <= order equal the continuous ones
        # (the spline's Fourier transform has zeros of order n+1 at 2 pi k).
        if o >= 2:
            assert abs((((nodes - xi) ** 2) * s).sum() - (o + 1) / 12.0) < 1e-14
        if o >= 3:
            assert abs((((nodes - xi) ** 3) * s).sum()) < 1e-14
        assert (s >= 0).all()
        assert np.count_nonzero(s) <= o + 1


@pytest.mark.parametrize("o", ORDERS)
def test_shape_continuity_and_support(o):
    for b in np.arange(-2.5, 2.51, 0.5):
        assert abs(S(o, b - 1e-12) - S(o, b + 1e-12)) < 1e-11
    assert S(o, (o + 1) / 2.0) == 0.0
    assert S(o, -(o + 1) / 2.0 - 1e-9) == 0.0
    assert S(o, 0.3) == S(o, -0.3)


def _yee_positions(n, comp, kind, dim=3):
    i, j, k = np.meshgrid(np.arange(n[0]), np.arange(n[1]), np.arange(n[2]), indexing="ij")
    sh = [0.0, 0.0, 0.0]
    for d in range(3):
        sh[d] = 0.5 if ((d == comp) if kind == "E" else (d != comp)) else 0.0
    if dim == 2:
        sh[1] = 0.0
    pos = [i + sh[0], j + sh[1], k + sh[2]]
    # flatten x-fastest: index i + n0 (j + n1 k)
    return [p.transpose(2, 1, 0).reshape(-1) for p in pos]


def _brute_gather(n, F, comp, kind, xi, o, dim=3):
    """Sum over every grid point and every periodic image in range."""
    P = _yee_positions(n, comp, kind, dim)
    tot = 0.0
    for c in range(F.shape[0]):
        for ox in (-n[0], 0, n[0]):
            for oy in ((-n[1], 0, n[1]) if dim == 3 else (0,)):
                for oz in (-n[2], 0, n[2]):
                    sx = S(o, xi[0] - (P[0][c] + ox))
                    sz = S(o, xi[2] - (P[2][c] + oz))
                    sy = S(o, xi[1] - (P[1][c] + oy)) if dim == 3 else 1.0
                    tot += F[c] * sx * sy * sz
    return tot


@pytest.mark.parametrize("o", ORDERS)
def test_gather_brute_force_tiny_grid(o):
    n = (4, 5, 3)
    g = oracle.make_grid(3, n, (1, 1, 1), 0.5, o)
    rng = np.random.default_rng(3)
    N = n[0] * n[1] * n[2]
    E = rng.standard_normal((3, N))
    B = rng.standard_normal((3, N))
    for _ in range(3):
        xi = rng.uniform(0, 1, 3) * np.array(n)
        Ep, Bp = oracle.gather(g, E, B, xi)
        for c in range(3):
            assert abs(Ep[c] - _brute_gather(n, E[c], c, "E", xi, o)) < 1e-12
            assert abs(Bp[c] - _brute_gather(n, B[c], c, "B", xi, o)) < 1e-12


@pytest.mark.parametrize("o", ORDERS)
def test_gather_uniform_and_linear_fields(o):
    n = (16, 16, 16)
    g = oracle.make_grid(3, n, (1, 1, 1), 0.5, o)
    N = n[0] * n[1] * n[2]
    rng = np.random.default_rng(4)
    E = np.zeros((3, N))
    B = np.zeros((3, N))
    a = rng.standard_normal(6)
    b = rng.standard_normal((6, 3))
    for c in range(3):
        PE = _yee_positions(n, c, "E")
        PB = _yee_positions(n, c, "B")
        E[c] = a[c] + sum(b[c, d] * PE[d] for d in range(3))
        B[c] = a[3 + c] + sum(b[3 + c, d] * PB[d] for d in range(3))
    for _ in range(20):
        xi = rng.uniform(4, 11, 3)      # window away from the periodic seam
        Ep, Bp = oracle.gather(g, E, B, xi)
        for c in range(3):
            assert abs(Ep[c] - (a[c] + b[c] @ xi)) < 1e-12
            assert abs(Bp[c] - (a[3 + c] + b[3 + c] @ xi)) < 1e-12


@pytest.mark.parametrize("o", ORDERS)
def test_gather_2d_equals_3d_with_one_y_cell(o):
    n = (6, 1, 5)
    g2 = oracle.make_grid(2, n, (1, 1, 1), 0.5, o)
    g3 = oracle.make_grid(3, n, (1, 1, 1), 0.5, o)
    rng = np.random.default_rng(5)
    E = rng.standard_normal((3, 30))
    B = rng.standard_normal((3, 30))
    for _ in range(10):
        xi = np.array([rng.uniform(0, 6), rng.uniform(0, 1), rng.uniform(0, 5)])
        E2, B2 = oracle.gather(g2, E, B, xi)
        E3, B3 = oracle.gather(g3, E, B, xi)
        assert np.allclose(E2, E3, rtol=0, atol=1e-13)
        assert np.allclose(B2, B3, rtol=0, atol=1e-13)


def test_rank_major_order_against_python_sorted():
    # brute force: sort by key (stable), rank within equal keys, then by
    # (tile, min(rank, 15)) keeping that order for ties
    rng = np.random.default_rng(21)
    cb = 3
    key = (rng.integers(0, 5, 400) << cb) | rng.integers(0, 8, 400)
    key = key.astype(np.int64)
    perm = oracle.rank_major(key, cb, 4)
    srt = sorted(range(len(key)), key=lambda i: key[i])
    rank = {}
    seen = {}
    for i in srt:
        rank[i] = min(seen.get(key[i], 0), 15)
        seen[key[i]] = seen.get(key[i], 0) + 1
    pos = {i: p for p, i in enumerate(srt)}
    expect = sorted(srt, key=lambda i: ((key[i] >> cb), rank[i], pos[i]))
    assert list(perm) == expect
    # consecutive particles of one rank in one tile sit in increasing cells
    t, c = key[perm] >> cb, key[perm] & 7
    r = np.array([rank[i] for i in perm])
    same = (t[1:] == t[:-1]) & (r[1:] == r[:-1])
    below_cap = same & (r[1:] < 15)
    assert np.all(c[1:][below_cap] > c[:-1][below_cap])
    assert np.all(c[1:][same] >= c[:-1][same])
