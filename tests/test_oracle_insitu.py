"""Pin of the oracle's per-layer moments: hand-computed sums for particles
placed in known layers (with the moving window's offset), and the layer
sums against the total weight and the (pinned) kinetic energy."""
import math

import numpy as np

import oracle
import pic_inputs as pi


class _S:
    def __init__(self, q, m, x, u, w):
        self.q, self.m = q, m
        self.x = np.ascontiguousarray(x, dtype=np.float64)
        self.u = np.ascontiguousarray(u, dtype=np.float64)
        self.w = np.ascontiguousarray(w, dtype=np.float64)


def test_hand_computed_layers():
    g = oracle.make_grid(3, (4, 4, 6), (1.0, 1.0, 1.0), 0.3, 1)
    x = np.array([[0.5, 1.5, 2.5], [0.5, 0.5, 0.5], [1.2, 1.9, 4.0]])
    u = np.array([[0.75, 0.0, 0.6], [0.0, 0.0, 0.8], [0.0, 2.4, 0.0]])
    w = np.array([2.0, 3.0, 5.0])
    sp = _S(-1.0, 4.0, x, u, w)
    m = oracle.slice_moments(g, sp)
    expect = np.zeros((6, 5))
    # layer 1: particles 0 (u = 3/4: gamma - 1 = 1/4) and 1 (u = 12/5: 8/5)
    expect[1] = [5.0, 2.0 * 0.75, 0.0, 3.0 * 2.4, 2.0 * 4.0 * 0.25 + 3.0 * 4.0 * 1.6]
    # layer 4: particle 2 (|u| = 1: gamma - 1 = sqrt 2 - 1)
    expect[4] = [5.0, 5.0 * 0.6, 5.0 * 0.8, 0.0, 5.0 * 4.0 * (math.sqrt(2.0) - 1.0)]
    np.testing.assert_allclose(m, expect, rtol=1e-14, atol=1e-15)
    # the window frame: offset 2 moves array layer k to frame layer k - 2
    m2 = oracle.slice_moments(g, sp, zoff=2)
    np.testing.assert_allclose(m2, np.roll(expect, -2, axis=0), rtol=1e-14, atol=1e-15)


def test_layer_sums_match_totals():
    wl = pi.uniform_box((6, 5, 9), 3, 0.05, 0.3, 2, 9950, "cpu", tile=(4, 4, 4))
    g = oracle.make_grid(3, (6, 5, 9), (1.0, 1.0, 1.0), 0.3, 2)
    sp = wl.species[0].numpy()
    m = oracle.slice_moments(g, sp)
    assert abs(m[:, 0].sum() - sp.w.sum()) < 1e-12 * sp.w.sum()
    ke = oracle.kinetic_energy(sp)
    assert abs(m[:, 4].sum() - ke) < 1e-12 * ke
    np.testing.assert_allclose(m[:, 1:4].sum(axis=0), (sp.w * sp.u).sum(axis=1), rtol=1e-10,
                               atol=1e-16)
