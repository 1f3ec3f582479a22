// Device-side arithmetic of one PIC particle update, shared by every kernel
// of libpic: B-spline weights in per-cell polynomial form, their divided
// differences (for a cancellation-free Esirkepov deposit), and the
// relativistic Boris rotation.  Written for gfx950 wave64; all functions are
// inlined into the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pic {

// ---------------------------------------------------------------- shapes
//
// The order-O B-spline S restricted to one "reference cell" [c', c'+1) of a
// node grid is, for each of the O+1 nodes c'+MLO+m it touches, a polynomial
// P_m of the in-cell coordinate f in [0, 1).  For odd O the reference cell
// is the cell holding the point; for even O it is the cell of the half-shifted
// coordinate xi + 1/2 (the spline's breakpoints sit at half-integers).
//   O = 1 (MLO = 0):  P0 = 1-f,  P1 = f
//   O = 2 (MLO = -1): P0 = (1-f)^2/2,  P1 = 1/2 + f - f^2,  P2 = f^2/2
//   O = 3 (MLO = -1): P0 = (1-f)^3/6,  P1 = 2/3 - f^2 + f^3/2,
//                     P2 = P1(1-f),    P3 = f^3/6
template <int O> struct Spline;

// Order 0 (the nearest node; the Galerkin gather of order-1 shapes along a
// staggered axis): reference cell of xi + 1/2, one node.
template <> struct Spline<0> {
    static constexpr int MLO = 0;
    static constexpr bool EVEN = true;
    template <typename R> __device__ static inline R P(int, R) { return R(1); }
    template <typename R> __device__ static inline R D(int, R, R) { return R(0); }
};

template <> struct Spline<1> {
    static constexpr int MLO = 0;
    static constexpr bool EVEN = false;
    template <typename R> __device__ static inline R P(int m, R f) {
        return m == 0 ? R(1) - f : f;
    }
    // divided difference [x, y] P_m
    template <typename R> __device__ static inline R D(int m, R, R) {
        return m == 0 ? R(-1) : R(1);
    }
};

template <> struct Spline<2> {
    static constexpr int MLO = -1;
    static constexpr bool EVEN = true;
    template <typename R> __device__ static inline R P(int m, R f) {
        if (m == 0) { R g = R(1) - f; return R(0.5) * g * g; }
        if (m == 1) return R(0.5) + f - f * f;
        return R(0.5) * f * f;
    }
    template <typename R> __device__ static inline R D(int m, R x, R y) {
        R h = R(0.5) * (x + y);
        if (m == 0) return h - R(1);
        if (m == 1) return R(1) - (x + y);
        return h;
    }
};

template <> struct Spline<3> {
    static constexpr int MLO = -1;
    static constexpr bool EVEN = false;
    template <typename R> __device__ static inline R P(int m, R f) {
        R g = R(1) - f;
        if (m == 0) return g * g * g * R(1.0 / 6.0);
        if (m == 1) return R(2.0 / 3.0) - f * f + R(0.5) * f * f * f;
        if (m == 2) return R(2.0 / 3.0) - g * g + R(0.5) * g * g * g;
        return f * f * f * R(1.0 / 6.0);
    }
    template <typename R> __device__ static inline R D(int m, R x, R y) {
        if (m == 0 || m == 2) {
            R gx = R(1) - x, gy = R(1) - y;
            R q = gx * gx + gx * gy + gy * gy;
            return m == 0 ? -q * R(1.0 / 6.0) : (gx + gy) - R(0.5) * q;
        }
        R q = x * x + x * y + y * y;
        return m == 1 ? R(0.5) * q - (x + y) : q * R(1.0 / 6.0);
    }
};

// Weights of one axis for a gather: nodes base .. base+O (array indices).
template <int O, typename R> struct GWin {
    int base;
    R w[O + 1];
};

// Reference cell of point (c, f) for nodes at i + st/2 (st = 0 or 1):
// the coordinate used is xi - st/2 (+1/2 for even orders).  The shift is
// applied to (c, f) without forming xi, so the FP32 split position keeps
// its precision: f-1/2 is exact for f >= 1/2; f+1/2 rounds only below it.
template <int O, typename R>
__device__ inline GWin<O, R> gather_window(int c, R f, int st) {
    using S = Spline<O>;
    // shift sigma = (EVEN ? +1/2 : 0) - st/2, one of -1/2, 0, +1/2
    int sig2 = (S::EVEN ? 1 : 0) - st;
    GWin<O, R> g;
    int cc = c;
    R ff = f;
    if (sig2 > 0) {
        if (f < R(0.5)) ff = f + R(0.5); else { ff = f - R(0.5); cc = c + 1; }
    } else if (sig2 < 0) {
        if (f >= R(0.5)) ff = f - R(0.5); else { ff = f + R(0.5); cc = c - 1; }
    }
    g.base = cc + S::MLO;
#pragma unroll
    for (int m = 0; m <= O; ++m) g.w[m] = S::template P<R>(m, ff);
    return g;
}

// Galerkin form along a staggered axis: the order-(O-1) window of the
// half-shifted nodes, placed in the O+1 slots of the order-O window (its
// nodes are a subset of them; the unused slot gets weight 0).
template <int O, typename R>
__device__ inline GWin<O, R> gather_window_galerkin(int c, R f) {
    GWin<O, R> g = gather_window<O, R>(c, f, 1);
    GWin<O - 1, R> l = gather_window<O - 1, R>(c, f, 1);
    const int sh = l.base - g.base;          // 0 or 1
#pragma unroll
    for (int m = 0; m <= O; ++m) {
        const R a = (m < O) ? l.w[m] : R(0);
        const R b = (m >= 1) ? l.w[m - 1] : R(0);
        g.w[m] = sh == 0 ? a : b;
    }
    return g;
}

// ---------------------------------------------------------------- deposit
//
// One axis of the Esirkepov window: O+2 nodes base .. base+O+1 covering the
// old and the new position (|displacement| < 1 cell), with the old weight
// S0 and the change dS = S1 - S0 of every node.  dS is formed without
// subtracting two nearly equal weights: within one reference cell
// P(f1) - P(f0) = (f1 - f0) [f0, f1]P, and across a cell face the move is
// split at the face, P(1) = P'(0) joining the two cells' polynomials.  The
// displacement f1 - f0 is taken from the unshifted offsets, so it carries a
// single rounding.
template <int O, typename R> struct DWin {
    int base;
    R S0[O + 2];
    R dS[O + 2];
};

template <int O, typename R>
__device__ inline DWin<O, R> deposit_window(int c0u, R f0u, int c1u, R f1u) {
    using S = Spline<O>;
    const int su = c1u - c0u;
    // Real displacement (identical in the shifted frame of even orders).
    R delta;
    if (su == 0) delta = f1u - f0u;
    else if (su > 0) delta = (R(1) - f0u) + f1u;
    else delta = -(f0u + (R(1) - f1u));
    int c0 = c0u, c1 = c1u;
    R f0 = f0u, f1 = f1u, bu0 = R(1) - f0u, bu1 = R(1) - f1u;
    if (S::EVEN) {
        if (f0u < R(0.5)) { f0 = f0u + R(0.5); bu0 = R(0.5) - f0u; }
        else { f0 = f0u - R(0.5); c0 = c0u + 1; bu0 = (R(1) - f0u) + R(0.5); }
        if (f1u < R(0.5)) { f1 = f1u + R(0.5); bu1 = R(0.5) - f1u; }
        else { f1 = f1u - R(0.5); c1 = c1u + 1; bu1 = (R(1) - f1u) + R(0.5); }
    }
    const int s = c1 - c0;
    DWin<O, R> d;
    if (s == 0) {
        d.base = c0 + S::MLO;
#pragma unroll
        for (int k = 0; k <= O; ++k) {
            d.S0[k] = S::template P<R>(k, f0);
            d.dS[k] = delta * S::template D<R>(k, f0, f1);
        }
        d.S0[O + 1] = R(0);
        d.dS[O + 1] = R(0);
    } else if (s > 0) {
        d.base = c0 + S::MLO;
#pragma unroll
        for (int k = 0; k <= O + 1; ++k) {
            R a = (k <= O) ? bu0 * S::template D<R>(k, f0, R(1)) : R(0);
            R b = (k >= 1) ? f1 * S::template D<R>(k - 1, R(0), f1) : R(0);
            d.S0[k] = (k <= O) ? S::template P<R>(k, f0) : R(0);
            d.dS[k] = a + b;
        }
    } else {
        d.base = c0 + S::MLO - 1;
#pragma unroll
        for (int k = 0; k <= O + 1; ++k) {
            R a = (k >= 1) ? -f0 * S::template D<R>(k - 1, R(0), f0) : R(0);
            R b = (k <= O) ? -bu1 * S::template D<R>(k, f1, R(1)) : R(0);
            d.S0[k] = (k >= 1) ? S::template P<R>(k - 1, f0) : R(0);
            d.dS[k] = a + b;
        }
    }
    return d;
}

// Node range [c - GL, c + GH] (relative to the particle's cell c) that the
// gather windows of all six Yee components can touch, and [c - JL, c + JH]
// that the deposit window can touch for any move of less than one cell.
template <int O> struct Halo;
template <> struct Halo<1> { static constexpr int GL = 1, GH = 1, JL = 1, JH = 2; };
template <> struct Halo<2> { static constexpr int GL = 1, GH = 2, JL = 2, JH = 3; };
template <> struct Halo<3> { static constexpr int GL = 2, GH = 2, JL = 2, JH = 3; };

// Gather node range of one field component along one axis, by its stagger
// st (0: integer points, 1: half-shifted): [c - lo, c + hi].
__host__ __device__ constexpr int gather_lo(int order, int st) {
    return order == 1 ? st : (order == 2 ? 1 : 1 + st);
}
__host__ __device__ constexpr int gather_hi(int order, int st) {
    return order == 1 ? 1 : (order == 2 ? 2 - st : 2);
}
// Stagger of field component comp (0..2: E, 3..5: B) along axis d.
__host__ __device__ constexpr int comp_stagger(int comp, int d) {
    return comp < 3 ? (comp == d ? 1 : 0) : (comp - 3 == d ? 0 : 1);
}

// ---------------------------------------------------------------- push

// Relativistic Boris rotation with h = q dt / (2 m).
template <typename R>
__device__ inline void boris(R h, const R E[3], const R B[3], R u[3]) {
    R um0 = u[0] + h * E[0], um1 = u[1] + h * E[1], um2 = u[2] + h * E[2];
    R gi = R(1) / sqrt(R(1) + um0 * um0 + um1 * um1 + um2 * um2);
    R t0 = h * B[0] * gi, t1 = h * B[1] * gi, t2 = h * B[2] * gi;
    R sc = R(2) / (R(1) + t0 * t0 + t1 * t1 + t2 * t2);
    R s0 = t0 * sc, s1 = t1 * sc, s2 = t2 * sc;
    R up0 = um0 + (um1 * t2 - um2 * t1);
    R up1 = um1 + (um2 * t0 - um0 * t2);
    R up2 = um2 + (um0 * t1 - um1 * t0);
    u[0] = um0 + (up1 * s2 - up2 * s1) + h * E[0];
    u[1] = um1 + (up2 * s0 - up0 * s2) + h * E[1];
    u[2] = um2 + (up0 * s1 - up1 * s0) + h * E[2];
}

// Relativistic pusher of Vay (Phys. Plasmas 15, 056701, 2008), with h =
// q dt / (2 m): u' = u + 2h (E + v x B / 2), tau = h B, then gamma^(n+1/2)
// from sigma = gamma'^2 - tau^2 and u* = u'.tau, t = tau / gamma^(n+1/2),
// u = (u' + (u'.t) t + u' x t) / (1 + t^2).  E + v x B vanishes exactly at
// the E x B drift velocity.
template <typename R>
__device__ inline void vay(R h, const R E[3], const R B[3], R u[3]) {
    const R gi0 = R(1) / sqrt(R(1) + u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
    const R v0 = u[0] * gi0, v1 = u[1] * gi0, v2 = u[2] * gi0;
    const R q2 = R(2) * h;
    const R up0 = u[0] + q2 * (E[0] + R(0.5) * (v1 * B[2] - v2 * B[1]));
    const R up1 = u[1] + q2 * (E[1] + R(0.5) * (v2 * B[0] - v0 * B[2]));
    const R up2 = u[2] + q2 * (E[2] + R(0.5) * (v0 * B[1] - v1 * B[0]));
    const R ta0 = h * B[0], ta1 = h * B[1], ta2 = h * B[2];
    const R tau2 = ta0 * ta0 + ta1 * ta1 + ta2 * ta2;
    const R us = up0 * ta0 + up1 * ta1 + up2 * ta2;
    const R sig = (R(1) + up0 * up0 + up1 * up1 + up2 * up2) - tau2;
    const R g1 = sqrt(R(0.5) * (sig + sqrt(sig * sig + R(4) * (tau2 + us * us))));
    const R t0 = ta0 / g1, t1 = ta1 / g1, t2 = ta2 / g1;
    const R sc = R(1) / (R(1) + t0 * t0 + t1 * t1 + t2 * t2);
    const R ut = up0 * t0 + up1 * t1 + up2 * t2;
    u[0] = sc * (up0 + ut * t0 + (up1 * t2 - up2 * t1));
    u[1] = sc * (up1 + ut * t1 + (up2 * t0 - up0 * t2));
    u[2] = sc * (up2 + ut * t2 + (up0 * t1 - up1 * t0));
}

// The momentum update of a species: Boris (pusher 0) or Vay (pusher 1).
template <typename R>
__device__ inline void push_momentum(int pusher, R h, const R E[3], const R B[3], R u[3]) {
    if (pusher == 1) vay<R>(h, E, B, u);
    else boris<R>(h, E, B, u);
}

__device__ inline int wrap_index(int i, int n) {
    // valid for i in (-n, 2n); callers guarantee it for n >= window width,
    // and use wrap_index_any otherwise.
    return i < 0 ? i + n : (i >= n ? i - n : i);
}

__device__ inline int wrap_index_any(int i, int n) {
    int r = i % n;
    return r < 0 ? r + n : r;
}

}  // namespace pic
