// Particle kernels of libpic: field gather, Boris push, position advance and
// Esirkepov current deposit, for one B-spline order (PIC_ORDER, set by the
// build: this file is compiled once per order).
//
// Three launch forms share one per-particle routine:
//   direct   one thread per particle; E/B read from global memory, J added
//            with global FP64 atomics.  Needs no sort.
//   tiled    one workgroup per (species, tile): the tile's E/B plus halo is
//            staged in LDS, J is accumulated in an LDS tile plus halo and
//            flushed once with global FP64 atomics.
//   batched  the tiled body driven by a persistent grid that pops
//            (species, tile, particle chunk) items from a global queue, so
//            tiles of very uneven population and many boxes share a launch.
// A particle whose cell has left its tile plus the staged margin since the
// last sort is appended to a straggler list by the tiled forms and updated
// through global memory by k_strag right after, so results never depend on
// how stale the sort is.
//
// Precision policies: F64 (FP64 positions, momenta, fields, LDS J) and
// Split (int32 cell + FP32 in-cell offset, FP32 momenta, fields, gather,
// push, deposit weights; the LDS current tile holds 64-bit fixed-point sums,
// flushed to FP64 J).
#include <type_traits>

#include "pic_dev.h"
#include "pic_math.h"
#include "pic_aux.h"

#if !defined(PIC_ORDER) || !defined(PIC_PREC) || !defined(PIC_PART)
#error "PIC_ORDER (1..3), PIC_PREC (0 FP64, 1 split) and PIC_PART (0..2) must be defined"
#endif

namespace pic {
namespace {

constexpr int O = PIC_ORDER;

#ifndef PIC_SKIP_ZERO_ATOMICS
#define PIC_SKIP_ZERO_ATOMICS 1
#endif
using H = Halo<O>;

// FP64 field values a thread loads before storing them to LDS (the FP64
// stage is copied through registers).
constexpr int STAGE_BATCH = 4;

__device__ inline void flag_range(int *err) { atomicOr(err, 1); }

// A workgroup-uniform descriptor (box, species) copied into scalar
// registers, word by word.  Read through a reference instead, its fields
// are reloaded with vector loads after every global store or atomic (the
// compiler cannot rule out aliasing), and each reload waits for all of the
// wave's stores and atomics in flight.
template <class T>
__device__ __forceinline__ T uniform_copy(const T &g) {
    static_assert(sizeof(T) % 4 == 0, "descriptor of whole words");
    int w[sizeof(T) / 4];
    __builtin_memcpy(w, &g, sizeof(T));
#pragma unroll
    for (int k = 0; k < (int)(sizeof(T) / 4); ++k) w[k] = __builtin_amdgcn_readfirstlane(w[k]);
    T r;
    __builtin_memcpy(&r, w, sizeof(T));
    return r;
}

// A pointer into device (global) memory that went through integer
// registers, declared global again so that accesses through it compile to
// global, not flat, memory instructions.
template <class T>
__device__ __forceinline__ T *global_ptr(T *p) {
    return (T *)(__attribute__((address_space(1))) T *)(unsigned long long)p;
}

__device__ __forceinline__ DevSpecies uniform_species(const DevSpecies &g) {
    DevSpecies s = uniform_copy(g);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        s.x[d] = global_ptr(s.x[d]);
        s.off[d] = global_ptr(s.off[d]);
        s.u[d] = global_ptr(s.u[d]);
        s.xo[d] = global_ptr(s.xo[d]);
        s.offo[d] = global_ptr(s.offo[d]);
    }
    s.cell = global_ptr(s.cell);
    s.w = global_ptr(s.w);
    s.cello = global_ptr(s.cello);
    s.carry = global_ptr(s.carry);
    s.strag = global_ptr(s.strag);
    s.tile_off = global_ptr(s.tile_off);
    return s;
}

// ------------------------------------------------------------ precision

struct F64 {
    using R = double;
    using FieldT = double;
    using Acc = double;
    static constexpr int PREC = 0;
    static constexpr int MAX_BLOCK = 512;    // tiled kernels: threads per workgroup
    // Old position from the species arrays or from scratch (all words read
    // before any is checked, so that the loads are in flight together).
    __device__ __forceinline__ static bool load(const DevBox &b, double *const xs[3], long long i,
                                int c[3], double f[3]) {
        double xv[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) xv[d] = (b.dim == 2 && d == 1) ? 0.0 : xs[d][i];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            if (b.dim == 2 && d == 1) { c[d] = 0; f[d] = 0.0; continue; }
            double x = xv[d];
            if (!(x >= 0.0 && x < (double)b.n[d])) return false;
            double fl = floor(x);
            c[d] = (int)fl;
            f[d] = x - fl;
        }
        return true;
    }
};

// floor(a / d) for 0 <= a < 2^31, 1 <= d < 2^31, from an FP64 reciprocal:
// the product is within one of the quotient, fixed by one correction step.
__device__ inline int div_exact(int a, int d, double inv_d) {
    int q = (int)((double)a * inv_d);
    int r = a - q * d;
    q += (r >= d) - (r < 0);
    return q;
}

// LDS current tile of the split form: 64-bit fixed-point integers with a
// per-tile power-of-two scale, summed with 64-bit integer LDS atomics and
// converted to FP64 by the flush.  Measured on gfx950 (wave instruction on
// distinct addresses): ds_add_f32 ~193 cycles per CU, ds_add_f64 ~8.5,
// ds_add_u64 ~6.4, and under 2-way bank conflicts 16.7 against 8.6.  Each
// contribution is an FP32 product truncated at 2^-30 of the tile's largest
// charge factor (finer than its own FP32 rounding), and integer sums do not
// depend on the order of the adds.
struct Split {
    using R = float;
    using FieldT = float;
    using Acc = long long;
    static constexpr int PREC = 1;
    static constexpr int MAX_BLOCK = 1024;   // 128 VGPRs: 16 waves per CU
    __device__ __forceinline__ static bool load(const DevBox &b, const int *cells, float *const offs[3],
                                long long i, int c[3], float f[3]) {
        // all words read before any is checked (loads in flight together)
        const int cell = cells[i];
        float ov[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) ov[d] = (b.dim == 2 && d == 1) ? 0.0f : offs[d][i];
        if (cell < 0 || (long long)cell >= b.ncells) return false;
        const int nx = b.n[0], nxy = b.n[0] * b.n[1];
        c[2] = div_exact(cell, nxy, b.inv_nxy);
        int r = cell - c[2] * nxy;
        c[1] = div_exact(r, nx, b.inv_nx);
        c[0] = r - c[1] * nx;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            if (b.dim == 2 && d == 1) { f[d] = 0.0f; continue; }
            const float v = ov[d];
            if (!(v >= 0.0f && v < 1.0f)) return false;
            f[d] = v;
        }
        return true;
    }
};

// ------------------------------------------------------------ accessors

template <typename T> struct GlobalField {
    static constexpr bool LDS = false;
    const T *F[6];
    int n0, n1, n2;
    bool any;
    __device__ inline T load(int comp, int i, int j, int k) const {
        if (any) {
            i = wrap_index_any(i, n0); j = wrap_index_any(j, n1); k = wrap_index_any(k, n2);
        } else {
            i = wrap_index(i, n0); j = wrap_index(j, n1); k = wrap_index(k, n2);
        }
        return F[comp][i + (long long)n0 * (j + (long long)n1 * k)];
    }
};

// The staged E/B tile: each component holds only the nodes its own gather
// stencil can reach (its extent differs by stagger), at its own offset.
template <typename T> struct LdsField {
    static constexpr bool LDS = true;
    const T *base;
    int off[6], o0[6], o1[6], o2[6], L0[6], L01[6];
    __device__ inline T load(int comp, int i, int j, int k) const {
        return *at(comp, i, j, k);
    }
    // Address of node (i, j, k) of a component; neighbours are reached by
    // adding the component's row (L0) and plane (L01) strides.
    __device__ inline const T *at(int comp, int i, int j, int k) const {
        return base + off[comp] + (i - o0[comp]) + L0[comp] * (j - o1[comp]) +
               L01[comp] * (k - o2[comp]);
    }
};

struct GlobalJ {
    static constexpr bool LDS = false;
    static constexpr bool FIXED = false;
    double *J[3];
    int n0, n1, n2;
    bool any;
    template <typename V>
    __device__ inline void add(int comp, int i, int j, int k, V v) const {
        if (any) {
            i = wrap_index_any(i, n0); j = wrap_index_any(j, n1); k = wrap_index_any(k, n2);
        } else {
            i = wrap_index(i, n0); j = wrap_index(j, n1); k = wrap_index(k, n2);
        }
        unsafeAtomicAdd(&J[comp][i + (long long)n0 * (j + (long long)n1 * k)], (double)v);
    }
};

// One addition into the LDS current tile: an FP64 atomic add, or, for a
// fixed-point tile, the contribution (already multiplied by the tile's
// scale, so |v| < 2^31) truncated to an integer and added as a 64-bit
// integer (ds_add_u64: cheaper than ds_add_f64 and far less sensitive to
// bank conflicts on gfx950, and order-independent).
template <typename A, typename V> __device__ __forceinline__ void lds_add(A *p, V v) {
    if constexpr (std::is_integral<A>::value) {
        // a plain conversion: one v_cvt_i32_f32 (rounds toward zero)
        const long long iv = (long long)(int)(float)v;
        atomicAdd((unsigned long long *)p, (unsigned long long)iv);
    } else {
        unsafeAtomicAdd(p, (A)v);
    }
}

template <typename A> struct LdsJ {
    static constexpr bool LDS = true;
    static constexpr bool FIXED = std::is_integral<A>::value;
    A *base;
    // components c = 0, 1, 2 at base + c * M012, rows of M0, M1 rows per
    // plane; N entries in all: J_z, whose edges along z end one node before
    // the region does, goes without its last plane
    int o0, o1, o2, M0, M1, M012, N;
    // fixed point: contributions are scaled by `scale` = 2^s before the
    // integer add, and the flush multiplies by `unscale` = 2^-s
    float scale;
    double unscale;
    __device__ inline A *at(int comp, int i, int j, int k) const {
        return base + comp * M012 + (i - o0) + M0 * ((j - o1) + M1 * (k - o2));
    }
    template <typename V>
    __device__ inline void add(int comp, int i, int j, int k, V v) const {
        lds_add(&base[comp * M012 + (i - o0) + M0 * ((j - o1) + M1 * (k - o2))], v);
    }
};

// ------------------------------------------------------------ gather

template <int DIM, typename R, class FA>
__device__ __forceinline__ R interp(const FA &fa, int comp, const GWin<O, R> &wx,
                           const GWin<O, R> &wy, const GWin<O, R> &wz) {
    R sum = R(0);
    if constexpr (FA::LDS) {
        const auto *p0 = fa.at(comp, wx.base, wy.base, wz.base);
        const int rs = fa.L0[comp], ps = fa.L01[comp];
        if (DIM == 3) {
#pragma unroll
            for (int kk = 0; kk <= O; ++kk) {
                R sy = R(0);
#pragma unroll
                for (int jj = 0; jj <= O; ++jj) {
                    const auto *r = p0 + kk * ps + jj * rs;
                    R sx = R(0);
#pragma unroll
                    for (int ii = 0; ii <= O; ++ii) sx += wx.w[ii] * (R)r[ii];
                    sy += wy.w[jj] * sx;
                }
                sum += wz.w[kk] * sy;
            }
        } else {
#pragma unroll
            for (int kk = 0; kk <= O; ++kk) {
                const auto *r = p0 + kk * ps;
                R sx = R(0);
#pragma unroll
                for (int ii = 0; ii <= O; ++ii) sx += wx.w[ii] * (R)r[ii];
                sum += wz.w[kk] * sx;
            }
        }
        return sum;
    }
    if (DIM == 3) {
        // from global memory one plane at a time: with every plane's loads
        // hoisted together the straggler kernels ran out of registers
#pragma unroll 1
        for (int kk = 0; kk <= O; ++kk) {
            R sy = R(0);
#pragma unroll
            for (int jj = 0; jj <= O; ++jj) {
                R sx = R(0);
#pragma unroll
                for (int ii = 0; ii <= O; ++ii)
                    sx += wx.w[ii] * (R)fa.load(comp, wx.base + ii, wy.base + jj, wz.base + kk);
                sy += wy.w[jj] * sx;
            }
            // the plane's weight by selects: indexing the window with the
            // loop counter would put it in scratch memory
            R wk = wz.w[0];
#pragma unroll
            for (int m = 1; m <= O; ++m) wk = kk == m ? wz.w[m] : wk;
            sum += wk * sy;
        }
    } else {
#pragma unroll
        for (int kk = 0; kk <= O; ++kk) {
            R sx = R(0);
#pragma unroll
            for (int ii = 0; ii <= O; ++ii)
                sx += wx.w[ii] * (R)fa.load(comp, wx.base + ii, 0, wz.base + kk);
            sum += wz.w[kk] * sx;
        }
    }
    return sum;
}

// Each component from its own Yee points: E_c is half-shifted along c,
// B_c along the two other axes.
// galerkin: along each axis where a component sits at half-integer points
// the shape is one order lower (the g1 windows are exactly those axes).
template <int DIM, typename R, class FA>
__device__ __forceinline__ void gather(const FA &fa, const int c[3], const R f[3], R E[3], R B[3],
                                       int galerkin) {
    GWin<O, R> g0[3], g1[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        if (DIM == 2 && d == 1) {
            g0[d].base = 0; g1[d].base = 0;
#pragma unroll
            for (int m = 0; m <= O; ++m) { g0[d].w[m] = R(0); g1[d].w[m] = R(0); }
            continue;
        }
        g0[d] = gather_window<O, R>(c[d], f[d], 0);
        if (galerkin) g1[d] = gather_window_galerkin<O, R>(c[d], f[d]);
        else g1[d] = gather_window<O, R>(c[d], f[d], 1);
    }
    E[0] = interp<DIM>(fa, 0, g1[0], g0[1], g0[2]);
    E[1] = interp<DIM>(fa, 1, g0[0], g1[1], g0[2]);
    E[2] = interp<DIM>(fa, 2, g0[0], g0[1], g1[2]);
    B[0] = interp<DIM>(fa, 3, g0[0], g1[1], g1[2]);
    B[1] = interp<DIM>(fa, 4, g1[0], g0[1], g1[2]);
    B[2] = interp<DIM>(fa, 5, g1[0], g1[1], g0[2]);
}

// ------------------------------------------------------------ deposit

// Esirkepov weights: W^x = dSx (S0y S0z + dSy S0z/2 + S0y dSz/2 + dSy dSz/3)
// and cyclically; J along an axis is the running sum of its W over the
// window, scaled by -q w / (dt * face area).  Since W^x factors into dSx_i
// times a (j, k) term, the running sum is (sum_{i'<=i} dSx_i') times that
// term: the scaled prefix sums are formed once per axis.  The last edge of
// each line carries the sum of all dS (zero) and is not written.
template <int DIM, typename R, class JA>
__device__ __forceinline__ void deposit(const JA &ja, const int c0[3], const R f0[3],
                               const int c1[3], const R f1[3], R cq[3], R vy) {
    constexpr int K = O + 2;
    DWin<O, R> wx = deposit_window<O, R>(c0[0], f0[0], c1[0], f1[0]);
    DWin<O, R> wz = deposit_window<O, R>(c0[2], f0[2], c1[2], f1[2]);
    const R third = R(1.0 / 3.0);
    // Line weights factor per axis: S0a S0b + (dSa S0b + S0a dSb)/2 + dSa dSb/3
    // = S0a (S0b + dSb/2) + dSa (S0b/2 + dSb/3) = S0a h_b + dSa q_b.
    R hx[K], qx[K], hz[K], qz[K];
#pragma unroll
    for (int m = 0; m < K; ++m) {
        hx[m] = wx.S0[m] + R(0.5) * wx.dS[m]; qx[m] = R(0.5) * wx.S0[m] + third * wx.dS[m];
        hz[m] = wz.S0[m] + R(0.5) * wz.dS[m]; qz[m] = R(0.5) * wz.S0[m] + third * wz.dS[m];
    }
    // Edges written per line: K-1 in general; when the particle stays in its
    // reference cell along that axis the window's last node carries no
    // weight, the flux through edge K-2 is sum(dS) = 0, and it is skipped.
    const int ex = (wx.S0[K - 1] == R(0) && wx.dS[K - 1] == R(0)) ? K - 2 : K - 1;
    const int ez = (wz.S0[K - 1] == R(0) && wz.dS[K - 1] == R(0)) ? K - 2 : K - 1;
    // The products handed to FP64 atomics are formed in FP64 from the prefix
    // sums and line weights, so no per-atomic conversion is needed; a
    // fixed-point LDS tile takes them in R (the charge factors arrive scaled).
    using A = typename std::conditional<JA::FIXED, R, double>::type;
    A px[K - 1], pz[K - 1];
    {
        R a = R(0), c = R(0);
#pragma unroll
        for (int i = 0; i < K - 1; ++i) {
            a += wx.dS[i]; px[i] = (A)(cq[0] * a);
            c += wz.dS[i]; pz[i] = (A)(cq[2] * c);
        }
    }
    if (DIM == 3) {
        DWin<O, R> wy = deposit_window<O, R>(c0[1], f0[1], c1[1], f1[1]);
        const int ey = (wy.S0[K - 1] == R(0) && wy.dS[K - 1] == R(0)) ? K - 2 : K - 1;
        R hy[K], qy[K];
#pragma unroll
        for (int m = 0; m < K; ++m) {
            hy[m] = wy.S0[m] + R(0.5) * wy.dS[m]; qy[m] = R(0.5) * wy.S0[m] + third * wy.dS[m];
        }
        A py[K - 1];
        {
            R a = R(0);
#pragma unroll
            for (int i = 0; i < K - 1; ++i) { a += wy.dS[i]; py[i] = (A)(cq[1] * a); }
        }
        if constexpr (JA::LDS) {
            // one base address per component; lines by uniform strides
            const int rs = ja.M0, ps = ja.M0 * ja.M1;
            auto *q0 = ja.at(0, wx.base, wy.base, wz.base);
            auto *q1 = ja.at(1, wx.base, wy.base, wz.base);
            auto *q2 = ja.at(2, wx.base, wy.base, wz.base);
#pragma unroll
            for (int k = 0; k < K; ++k) {
#pragma unroll
                for (int j = 0; j < K; ++j) {
                    R t = wy.S0[j] * hz[k] + wy.dS[j] * qz[k];
                    if (t == R(0)) continue;
                    auto *line = q0 + k * ps + j * rs;
#pragma unroll
                    for (int i = 0; i < K - 1; ++i)
                        if (i < ex) lds_add(line + i, px[i] * (A)t);
                }
            }
#pragma unroll
            for (int k = 0; k < K; ++k) {
#pragma unroll
                for (int i = 0; i < K; ++i) {
                    R t = wz.S0[k] * hx[i] + wz.dS[k] * qx[i];
                    if (t == R(0)) continue;
                    auto *line = q1 + k * ps + i;
#pragma unroll
                    for (int j = 0; j < K - 1; ++j)
                        if (j < ey) lds_add(line + j * rs, py[j] * (A)t);
                }
            }
#pragma unroll
            for (int j = 0; j < K; ++j) {
#pragma unroll
                for (int i = 0; i < K; ++i) {
                    R t = wx.S0[i] * hy[j] + wx.dS[i] * qy[j];
                    if (t == R(0)) continue;
                    auto *line = q2 + j * rs + i;
#pragma unroll
                    for (int k = 0; k < K - 1; ++k)
                        if (k < ez) lds_add(line + k * ps, pz[k] * (A)t);
                }
            }
            return;
        }
#pragma unroll
        for (int k = 0; k < K; ++k) {
#pragma unroll
            for (int j = 0; j < K; ++j) {
                R t = wy.S0[j] * hz[k] + wy.dS[j] * qz[k];
                if (t == R(0)) continue;
#pragma unroll
                for (int i = 0; i < K - 1; ++i)
                    if (i < ex) ja.add(0, wx.base + i, wy.base + j, wz.base + k, px[i] * (A)t);
            }
        }
#pragma unroll
        for (int k = 0; k < K; ++k) {
#pragma unroll
            for (int i = 0; i < K; ++i) {
                R t = wz.S0[k] * hx[i] + wz.dS[k] * qx[i];
                if (t == R(0)) continue;
#pragma unroll
                for (int j = 0; j < K - 1; ++j)
                    if (j < ey) ja.add(1, wx.base + i, wy.base + j, wz.base + k, py[j] * (A)t);
            }
        }
#pragma unroll
        for (int j = 0; j < K; ++j) {
#pragma unroll
            for (int i = 0; i < K; ++i) {
                R t = wx.S0[i] * hy[j] + wx.dS[i] * qy[j];
                if (t == R(0)) continue;
#pragma unroll
                for (int k = 0; k < K - 1; ++k)
                    if (k < ez) ja.add(2, wx.base + i, wy.base + j, wz.base + k, pz[k] * (A)t);
            }
        }
    } else {
        if constexpr (JA::LDS) {
            const int ps = ja.M0 * ja.M1;
            auto *q0 = ja.at(0, wx.base, 0, wz.base);
            auto *q1 = ja.at(1, wx.base, 0, wz.base);
            auto *q2 = ja.at(2, wx.base, 0, wz.base);
#pragma unroll
            for (int k = 0; k < K; ++k) {
                R t = hz[k];
                if (t == R(0)) continue;
#pragma unroll
                for (int i = 0; i < K - 1; ++i)
                    if (i < ex) lds_add(q0 + k * ps + i, px[i] * (A)t);
            }
#pragma unroll
            for (int i = 0; i < K; ++i) {
                R t = hx[i];
                if (t == R(0)) continue;
#pragma unroll
                for (int k = 0; k < K - 1; ++k)
                    if (k < ez) lds_add(q2 + k * ps + i, pz[k] * (A)t);
            }
            const A cy = (A)(cq[1] * vy);
#pragma unroll
            for (int k = 0; k < K; ++k) {
#pragma unroll
                for (int i = 0; i < K; ++i) {
                    R a = wx.S0[i] * hz[k] + wx.dS[i] * qz[k];
                    if (a != R(0)) lds_add(q1 + k * ps + i, cy * (A)a);
                }
            }
            return;
        }
#pragma unroll
        for (int k = 0; k < K; ++k) {
            R t = hz[k];
            if (t == R(0)) continue;
#pragma unroll
            for (int i = 0; i < K - 1; ++i)
                if (i < ex) ja.add(0, wx.base + i, 0, wz.base + k, px[i] * (A)t);
        }
#pragma unroll
        for (int i = 0; i < K; ++i) {
            R t = hx[i];
            if (t == R(0)) continue;
#pragma unroll
            for (int k = 0; k < K - 1; ++k)
                if (k < ez) ja.add(2, wx.base + i, 0, wz.base + k, pz[k] * (A)t);
        }
        const A cy = (A)(cq[1] * vy);
#pragma unroll
        for (int k = 0; k < K; ++k) {
#pragma unroll
            for (int i = 0; i < K; ++i) {
                R a = wx.S0[i] * hz[k] + wx.dS[i] * qz[k];
                if (a != R(0)) ja.add(1, wx.base + i, 0, wz.base + k, cy * (A)a);
            }
        }
    }
}

// ------------------------------------------------------------ one particle

// A tile's cells [t0, t0 + te) plus the staged margin of mg[d] cells per axis, so a
// particle that drifted up to mg cells out of its tile since the last sort
// still gathers and deposits through LDS.  In 2D the y range is the single
// cell 0 and always holds.
struct Tile {
    int t0[3], te[3];
    int mg[3];
    __device__ inline bool holds(const int c[3]) const {
        return c[0] >= t0[0] - mg[0] && c[0] < t0[0] + te[0] + mg[0] &&
               c[1] >= t0[1] - mg[1] && c[1] < t0[1] + te[1] + mg[1] &&
               c[2] >= t0[2] - mg[2] && c[2] < t0[2] + te[2] + mg[2];
    }
};

// One particle update.  TILED: gather and deposit through the work item's
// LDS tiles; a particle whose cell lies outside the tile plus margin is not
// updated here but appended to its species' straggler list (processed by
// k_strag right after).  Not TILED: global arrays with wrapped indices.
template <int DIM, class P, int MODE, bool TILED, class FL, class JL>
__device__ __forceinline__ void particle(const DevBox &b, const DevSpecies &sp, long long i,
                                         const DevFields &gf, const Tile *tile, const FL *lf,
                                         const JL *lj, int *err, int *strag_count) {
    using R = typename P::R;
    using FT = typename P::FieldT;
    int c0[3], c1[3];
    R f0[3], f1[3], u[3];
    bool ok;
    const bool any = b.small != 0;
    if (MODE & MODE_PUSH) {
        if constexpr (P::PREC == 0) ok = P::load(b, sp.x, i, c0, f0);
        else ok = P::load(b, sp.cell, sp.off, i, c0, f0);
    } else {
        if constexpr (P::PREC == 0) ok = P::load(b, sp.xo, i, c0, f0);
        else ok = P::load(b, sp.cello, sp.offo, i, c0, f0);
    }
    if (!ok) { flag_range(err); return; }
    if constexpr (TILED) {
        if (!tile->holds(c0)) {
            sp.strag[atomicAdd(strag_count, 1)] = (int)i;
            return;
        }
    }
    const R *ua[3] = {(const R *)sp.u[0], (const R *)sp.u[1], (const R *)sp.u[2]};
    u[0] = ua[0][i]; u[1] = ua[1][i]; u[2] = ua[2][i];
    const R dt = (R)b.dt;
    if (MODE & MODE_PUSH) {
        R E[3], B[3];
        if constexpr (TILED) {
            gather<DIM, R>(*lf, c0, f0, E, B, sp.galerkin);
        } else {
            GlobalField<FT> g;
#pragma unroll
            for (int cc = 0; cc < 3; ++cc) {
                g.F[cc] = (const FT *)gf.E[cc] + b.cell_base;
                g.F[cc + 3] = (const FT *)gf.B[cc] + b.cell_base;
            }
            g.n0 = b.n[0]; g.n1 = b.n[1]; g.n2 = b.n[2]; g.any = any;
            gather<DIM, R>(g, c0, f0, E, B, sp.galerkin);
        }
        const R h = (R)(sp.q * b.dt / (2.0 * sp.m));
        push_momentum<R>(sp.pusher, h, E, B, u);
        const R gi = R(1) / sqrt(R(1) + u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
        R disp[3];
        bool good = true;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            disp[d] = (DIM == 2 && d == 1) ? R(0) : dt * u[d] * gi / (R)b.dx[d];
            // below one cell with margin for rounding, so the deposit window
            // always spans at most O+2 nodes per axis
            good = good && (fabs(disp[d]) < R(0.999));
        }
        if (!good) {
            // Flag and leave the particle where it is; a later deposit of
            // this push sees no motion (and so adds no current).
            flag_range(err);
            if (MODE == MODE_PUSH) {
                if constexpr (P::PREC == 0) {
#pragma unroll
                    for (int d = 0; d < 3; ++d)
                        if (!(DIM == 2 && d == 1)) sp.xo[d][i] = (double)c0[d] + f0[d];
                } else {
                    sp.cello[i] = sp.cell[i];
#pragma unroll
                    for (int d = 0; d < 3; ++d)
                        if (!(DIM == 2 && d == 1)) sp.offo[d][i] = f0[d];
                    sp.carry[i] = 0x15;      // (0 + 1) per axis: no cell change
                }
            }
            return;
        }
        // new position (cell + offset, unwrapped cell index)
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            if (DIM == 2 && d == 1) { c1[d] = 0; f1[d] = R(0); continue; }
            if constexpr (P::PREC == 0) {
                double x1 = ((double)c0[d] + f0[d]) + disp[d];
                double fl = floor(x1);
                c1[d] = (int)fl;
                f1[d] = x1 - fl;
            } else {
                float fr = f0[d] + disp[d];
                if (fr >= 1.0f) { c1[d] = c0[d] + 1; f1[d] = fr - 1.0f; }
                else if (fr < 0.0f) {
                    c1[d] = c0[d] - 1; f1[d] = fr + 1.0f;
                    if (f1[d] == 1.0f) { f1[d] = 0.0f; c1[d] = c0[d]; }
                } else { c1[d] = c0[d]; f1[d] = fr; }
            }
        }
        if (MODE == MODE_PUSH) {
            // keep x^n for the deposit; store x^(n+1) and u^(n+1/2)
            R *uo[3] = {(R *)sp.u[0], (R *)sp.u[1], (R *)sp.u[2]};
#pragma unroll
            for (int d = 0; d < 3; ++d) uo[d][i] = u[d];
            if constexpr (P::PREC == 0) {
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    if (DIM == 2 && d == 1) continue;
                    sp.xo[d][i] = (double)c0[d] + f0[d];
                    sp.x[d][i] = (double)c1[d] + f1[d];           // unwrapped
                }
            } else {
                sp.cello[i] = sp.cell[i];
                int carry = 0;
                int cw[3];
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    cw[d] = c1[d];
                    if (DIM == 2 && d == 1) continue;
                    sp.offo[d][i] = f0[d];
                    sp.off[d][i] = f1[d];
                    carry |= (c1[d] - c0[d] + 1) << (2 * d);
                    cw[d] = wrap_index(c1[d], b.n[d]);
                }
                sp.carry[i] = carry;
                sp.cell[i] = cw[0] + b.n[0] * (cw[1] + b.n[1] * cw[2]);
            }
            return;
        }
    } else {
        // DEPOSIT only: x^(n+1) from the species arrays
        if constexpr (P::PREC == 0) {
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                if (DIM == 2 && d == 1) { c1[d] = 0; f1[d] = 0.0; continue; }
                double x1 = sp.x[d][i];
                double fl = floor(x1);
                c1[d] = (int)fl;
                f1[d] = x1 - fl;
                if (c1[d] - c0[d] > 1 || c0[d] - c1[d] > 1 || !(x1 == x1)) { flag_range(err); return; }
            }
        } else {
            const int carry = sp.carry[i];
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                if (DIM == 2 && d == 1) { c1[d] = 0; f1[d] = 0.0f; continue; }
                const int sd = ((carry >> (2 * d)) & 3) - 1;
                if (sd > 1) { flag_range(err); return; }
                c1[d] = c0[d] + sd;
                f1[d] = sp.off[d][i];
                if (!(f1[d] >= 0.0f && f1[d] < 1.0f)) { flag_range(err); return; }
            }
        }
    }
    // ---- deposit x^n -> x^(n+1)
    {
        const R wgt = ((const R *)sp.w)[i];
        const double dV = b.dx[0] * b.dx[1] * b.dx[2];
        R cq[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) cq[d] = (R)(-sp.q * b.dx[d] / (b.dt * dV)) * wgt;
        R vy = R(0);
        if (DIM == 2) {
            // out-of-plane current q w v_y / dV
            const R gi = R(1) / sqrt(R(1) + u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
            cq[1] = (R)(sp.q / dV) * wgt;
            vy = u[1] * gi;
        }
        if constexpr (TILED) {
            if constexpr (JL::FIXED) {
#pragma unroll
                for (int d = 0; d < 3; ++d) cq[d] *= lj->scale;
            }
            deposit<DIM, R>(*lj, c0, f0, c1, f1, cq, vy);
        } else {
            GlobalJ g;
#pragma unroll
            for (int cc = 0; cc < 3; ++cc) g.J[cc] = gf.J[cc] + b.cell_base;
            g.n0 = b.n[0]; g.n1 = b.n[1]; g.n2 = b.n[2]; g.any = any;
            deposit<DIM, R>(g, c0, f0, c1, f1, cq, vy);
        }
    }
    // ---- store wrapped x^(n+1) (and u)
    if (MODE == MODE_FUSED) {
        R *uo[3] = {(R *)sp.u[0], (R *)sp.u[1], (R *)sp.u[2]};
#pragma unroll
        for (int d = 0; d < 3; ++d) uo[d][i] = u[d];
    }
    if constexpr (P::PREC == 0) {
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            if (DIM == 2 && d == 1) continue;
            double x = (double)c1[d] + f1[d];
            const double L = (double)b.n[d];
            if (x >= L) x -= L;
            if (x < 0.0) x += L;
            if (x >= L) x = 0.0;
            sp.x[d][i] = x;
        }
    } else if (MODE == MODE_FUSED) {
        int cw[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            if (DIM == 2 && d == 1) { cw[d] = 0; continue; }
            cw[d] = wrap_index(c1[d], b.n[d]);
            sp.off[d][i] = f1[d];
        }
        sp.cell[i] = cw[0] + b.n[0] * (cw[1] + b.n[1] * cw[2]);
    }
}

// ------------------------------------------------------------ converged fused path
//
// The fused tiled kernels run every lane of a wave through the whole update
// (lanes without a particle carry weight 0), so that the four lanes of a
// quad can pool their deposit values with DPP before one of them issues the
// LDS atomic: with the particles of a cell in consecutive lanes (lane stride
// 1, ppc a multiple of 4) a quad shares one stencil, and the LDS sees a
// quarter of the atomic lanes.

template <int CTRL> __device__ inline int dpp_i(int v) {
    return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, true);
}
template <int CTRL> __device__ inline float dpp(float v) {
    return __int_as_float(dpp_i<CTRL>(__float_as_int(v)));
}
template <int CTRL> __device__ inline double dpp(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = dpp_i<CTRL>((int)(b & 0xffffffffll));
    const int hi = dpp_i<CTRL>((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}
// quad_perm selectors: [1,0,3,2], [2,3,0,1], [0,0,0,0]
constexpr int QP_SWAP1 = 0xB1, QP_SWAP2 = 0x4E, QP_LANE0 = 0x00;

template <typename T> __device__ inline T quad_sum(T v) {
    v += dpp<QP_SWAP1>(v);
    v += dpp<QP_SWAP2>(v);
    return v;
}

// Reduce-scatter over a quad: lane r (r = lane mod 4) returns the sum over
// the quad's lanes of their v[r].  Two exchange steps: lanes r and r^2 swap
// the half of the values the other keeps, then lanes r and r^1 do the same.
template <typename T> __device__ inline T quad_reduce_scatter(const T v[4]) {
    const int r = threadIdx.x & 3;
    const bool b1 = (r & 2) != 0, b0 = (r & 1) != 0;
    const T sendA = b1 ? v[0] : v[2], sendB = b1 ? v[1] : v[3];
    const T keepA = b1 ? v[2] : v[0], keepB = b1 ? v[3] : v[1];
    const T a0 = keepA + dpp<QP_SWAP2>(sendA);
    const T a1 = keepB + dpp<QP_SWAP2>(sendB);
    const T send = b0 ? a0 : a1;
    return (b0 ? a1 : a0) + dpp<QP_SWAP1>(send);
}

__device__ inline bool wave_any(bool p) { return __ballot(p) != 0ull; }

// Esirkepov deposit into the LDS current tile with every lane active.
// QUAD: a quad whose four lanes share one window pools each line: lane r
// adds the quad's sum of edge r.  Other quads add their own non-zero values,
// each lane starting at a different edge.
template <int DIM, bool QUAD, typename R, class JA>
__device__ __forceinline__ void deposit_converged(const JA &ja, const int c0[3], const R f0[3],
                                                  const int c1[3], const R f1[3], const R cq[3],
                                                  R vy, bool valid) {
    using A = typename std::remove_pointer<decltype(ja.base)>::type;
    constexpr int K = O + 2;
    DWin<O, R> wx = deposit_window<O, R>(c0[0], f0[0], c1[0], f1[0]);
    DWin<O, R> wz = deposit_window<O, R>(c0[2], f0[2], c1[2], f1[2]);
    DWin<O, R> wy;
    if (DIM == 3) wy = deposit_window<O, R>(c0[1], f0[1], c1[1], f1[1]);
    const R third = R(1.0 / 3.0);
    // factored line weights, as in deposit()
    R hx[K], qx[K], hy[K], qy[K], hz[K], qz[K];
#pragma unroll
    for (int m = 0; m < K; ++m) {
        hx[m] = wx.S0[m] + R(0.5) * wx.dS[m]; qx[m] = R(0.5) * wx.S0[m] + third * wx.dS[m];
        hz[m] = wz.S0[m] + R(0.5) * wz.dS[m]; qz[m] = R(0.5) * wz.S0[m] + third * wz.dS[m];
        if (DIM == 3) {
            hy[m] = wy.S0[m] + R(0.5) * wy.dS[m]; qy[m] = R(0.5) * wy.S0[m] + third * wy.dS[m];
        } else {
            hy[m] = R(0); qy[m] = R(0);
        }
    }
    const bool lastx = !(wx.S0[K - 1] == R(0) && wx.dS[K - 1] == R(0));
    const bool lastz = !(wz.S0[K - 1] == R(0) && wz.dS[K - 1] == R(0));
    const bool lasty = DIM == 3 && !(wy.S0[K - 1] == R(0) && wy.dS[K - 1] == R(0));
    const int exu = wave_any(lastx) ? K - 1 : K - 2;
    const int ezu = wave_any(lastz) ? K - 1 : K - 2;
    const int eyu = wave_any(lasty) ? K - 1 : K - 2;
    // Prefix sums of a line's edge values, scaled by the particle's charge
    // factor.  Without quad pooling they are kept in the LDS accumulation
    // type, so a line's products need one conversion (of t), not one per
    // edge; pooled quads combine them in R first.
    using PV = typename std::conditional<QUAD || JA::FIXED, R, A>::type;
    PV px[K - 1], py[K - 1], pz[K - 1];
    {
        R a = R(0), b = R(0), c = R(0);
#pragma unroll
        for (int i = 0; i < K - 1; ++i) {
            a += wx.dS[i]; px[i] = (i < K - 2 || lastx) ? (PV)(cq[0] * a) : PV(0);
            c += wz.dS[i]; pz[i] = (i < K - 2 || lastz) ? (PV)(cq[2] * c) : PV(0);
            if (DIM == 3) { b += wy.dS[i]; py[i] = (i < K - 2 || lasty) ? (PV)(cq[1] * b) : PV(0); }
        }
    }
    bool pool = false;
    if constexpr (QUAD) {
        const int by = DIM == 3 ? wy.base : 0;
        bool same = valid && wx.base == dpp_i<QP_LANE0>(wx.base) && by == dpp_i<QP_LANE0>(by) &&
                    wz.base == dpp_i<QP_LANE0>(wz.base);
        int f = same ? 1 : 0;
        f &= dpp_i<QP_SWAP1>(f);
        f &= dpp_i<QP_SWAP2>(f);
        pool = f != 0;
    }
    const bool lead = (threadIdx.x & 3) == 0;
    // One line of up to 4 edges, `ne` of them written (wave-uniform), at
    // addresses base + e * stride.  Pooled quads: lane r adds edge r.
    // rim: the line lies on the last node of the window along one of its two
    // transverse axes, where a lane whose particle stays in its cell has a
    // zero weight.
    auto line_put = [&](A *base, int stride, const PV *pv, R t, int ne, bool rim) {
        PV v[4];
        const PV tv = (PV)t;
#pragma unroll
        for (int e = 0; e < 4; ++e) v[e] = (e < K - 1 && e < ne) ? pv[e] * tv : PV(0);
        if constexpr (QUAD) {
            const R sc = quad_reduce_scatter(v);
            const int r = threadIdx.x & 3;
            if (pool) {
                if (r < ne) lds_add(base + r * stride, sc);
            } else {
                // Lane r of the quad adds edge (e + r) mod NE at step e, NE =
                // K - 1 edges per line: for NE = 4 lanes of one quad that
                // share a cell never hit one address at once (NE < 4: at
                // most lanes r and r + NE do).
                constexpr int NE = K - 1;
#pragma unroll
                for (int e = 0; e < NE; ++e) {
                    const int ed = (e + r) % NE;
                    const R x = ed == 0 ? v[0] : ed == 1 ? v[1] : ed == 2 ? v[2] : v[3];
                    if (ed < ne && x != R(0)) lds_add(base + ed * stride, x);
                }
            }
        } else {
#pragma unroll
            for (int e = 0; e < K - 1; ++e) {
#if PIC_SKIP_ZERO_ATOMICS
                // Zero values are skipped where they are common: on rim lines
                // and on the last edge of a line (zero for a particle that
                // stays in its cell along the line).  With the fixed-point
                // tile the other edges are added without a test (measured
                // faster on C5: the test and its exec-mask branch cost more
                // than the rare zero adds); the FP64 tile keeps the test.
                const bool test = !JA::FIXED || rim || e == K - 2;
                if (e < ne && (!test || v[e] != PV(0))) lds_add(base + e * stride, v[e]);
#else
                if (e < ne) lds_add(base + e * stride, v[e]);
#endif
            }
        }
    };
    auto put = [&](A *addr, R v) {
        if constexpr (QUAD) {
            const R s = quad_sum(v);
            if (pool) {
                if (lead) lds_add(addr, s);
            } else if (v != R(0)) {
                lds_add(addr, v);
            }
        } else {
            if (v != R(0)) lds_add(addr, v);
        }
    };
    const int rs = ja.M0, ps = ja.M0 * ja.M1;
    if (DIM == 3) {
        A *q0 = ja.at(0, wx.base, wy.base, wz.base);
        A *q1 = ja.at(1, wx.base, wy.base, wz.base);
        A *q2 = ja.at(2, wx.base, wy.base, wz.base);
#pragma unroll
        for (int k = 0; k < K; ++k) {
#pragma unroll
            for (int j = 0; j < K; ++j) {
                R t = wy.S0[j] * hz[k] + wy.dS[j] * qz[k];
                if (!wave_any(t != R(0))) continue;
                line_put(q0 + k * ps + j * rs, 1, px, t, exu, j == K - 1 || k == K - 1);
            }
        }
#pragma unroll
        for (int k = 0; k < K; ++k) {
#pragma unroll
            for (int i = 0; i < K; ++i) {
                R t = wz.S0[k] * hx[i] + wz.dS[k] * qx[i];
                if (!wave_any(t != R(0))) continue;
                line_put(q1 + k * ps + i, rs, py, t, eyu, i == K - 1 || k == K - 1);
            }
        }
#pragma unroll
        for (int j = 0; j < K; ++j) {
#pragma unroll
            for (int i = 0; i < K; ++i) {
                R t = wx.S0[i] * hy[j] + wx.dS[i] * qy[j];
                if (!wave_any(t != R(0))) continue;
                line_put(q2 + j * rs + i, ps, pz, t, ezu, i == K - 1 || j == K - 1);
            }
        }
    } else {
        A *q0 = ja.at(0, wx.base, 0, wz.base);
        A *q1 = ja.at(1, wx.base, 0, wz.base);
        A *q2 = ja.at(2, wx.base, 0, wz.base);
#pragma unroll
        for (int k = 0; k < K; ++k) {
            R t = hz[k];
            if (!wave_any(t != R(0))) continue;
            line_put(q0 + k * ps, 1, px, t, exu, k == K - 1);
        }
#pragma unroll
        for (int i = 0; i < K; ++i) {
            R t = hx[i];
            if (!wave_any(t != R(0))) continue;
            line_put(q2 + i, ps, pz, t, ezu, i == K - 1);
        }
        const R cy = cq[1] * vy;
#pragma unroll
        for (int k = 0; k < K; ++k) {
#pragma unroll
            for (int i = 0; i < K; ++i) {
                R a = wx.S0[i] * hz[k] + wx.dS[i] * qz[k];
                if (!wave_any(a != R(0))) continue;
                put(q1 + k * ps + i, cy * a);
            }
        }
    }
}

// Fused gather / push / advance / deposit / wrap of one slot of a tiled work
// item, with every lane active.  `have` is false for slots past the item's
// end; such lanes, particles with invalid input and particles outside the
// tile plus margin (queued as stragglers) compute on a dummy position at the
// tile origin with weight 0 and store nothing.
template <int DIM, class P, bool QUAD, class FL, class JL>
__device__ __forceinline__ void particle_converged(const DevBox &b, const DevSpecies &sp,
                                                   long long i, bool have, const Tile &tile,
                                                   const FL &lf, const JL &lj, int *err,
                                                   int *strag_count) {
    using R = typename P::R;
    int c0[3], c1[3];
    R f0[3], f1[3], u[3] = {R(0), R(0), R(0)};
    R wraw = R(0);
    bool valid = have;
    if (valid) {
        // momentum and weight are read with the position, before any check,
        // so that all of the slot's loads are in flight together
        const R *ua[3] = {(const R *)sp.u[0], (const R *)sp.u[1], (const R *)sp.u[2]};
        u[0] = ua[0][i]; u[1] = ua[1][i]; u[2] = ua[2][i];
        wraw = ((const R *)sp.w)[i];
        bool ok;
        if constexpr (P::PREC == 0) ok = P::load(b, sp.x, i, c0, f0);
        else ok = P::load(b, sp.cell, sp.off, i, c0, f0);
        if (!ok) { flag_range(err); valid = false; }
    }
    if (valid && !tile.holds(c0)) {
        sp.strag[atomicAdd(strag_count, 1)] = (int)i;
        valid = false;
    }
    if (!valid) {
#pragma unroll
        for (int d = 0; d < 3; ++d) { c0[d] = tile.t0[d]; f0[d] = R(0); u[d] = R(0); }
    }
    R E[3], B[3];
    gather<DIM, R>(lf, c0, f0, E, B, sp.galerkin);
    const R dt = (R)b.dt;
    const R h = (R)(sp.q * b.dt / (2.0 * sp.m));
    push_momentum<R>(sp.pusher, h, E, B, u);
    const R gi = R(1) / sqrt(R(1) + u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
    R disp[3];
    bool good = true;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        disp[d] = (DIM == 2 && d == 1) ? R(0) : dt * u[d] * gi / (R)b.dx[d];
        good = good && (fabs(disp[d]) < R(0.999));
    }
    if (valid && !good) { flag_range(err); valid = false; }
    if (!valid) {
#pragma unroll
        for (int d = 0; d < 3; ++d) disp[d] = R(0);
    }
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        if (DIM == 2 && d == 1) { c1[d] = 0; f1[d] = R(0); continue; }
        if constexpr (P::PREC == 0) {
            double x1 = ((double)c0[d] + f0[d]) + disp[d];
            double fl = floor(x1);
            c1[d] = (int)fl;
            f1[d] = x1 - fl;
        } else {
            float fr = f0[d] + disp[d];
            if (fr >= 1.0f) { c1[d] = c0[d] + 1; f1[d] = fr - 1.0f; }
            else if (fr < 0.0f) {
                c1[d] = c0[d] - 1; f1[d] = fr + 1.0f;
                if (f1[d] == 1.0f) { f1[d] = 0.0f; c1[d] = c0[d]; }
            } else { c1[d] = c0[d]; f1[d] = fr; }
        }
    }
    const R wgt = valid ? wraw : R(0);
    const double dV = b.dx[0] * b.dx[1] * b.dx[2];
    R cq[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) cq[d] = (R)(-sp.q * b.dx[d] / (b.dt * dV)) * wgt;
    R vy = R(0);
    if (DIM == 2) {
        cq[1] = (R)(sp.q / dV) * wgt;
        vy = u[1] * gi;
    }
    if constexpr (JL::FIXED) {
#pragma unroll
        for (int d = 0; d < 3; ++d) cq[d] *= lj.scale;
    }
    deposit_converged<DIM, QUAD, R>(lj, c0, f0, c1, f1, cq, vy, valid);
    if (!valid) return;
    R *uo[3] = {(R *)sp.u[0], (R *)sp.u[1], (R *)sp.u[2]};
#pragma unroll
    for (int d = 0; d < 3; ++d) uo[d][i] = u[d];
    if constexpr (P::PREC == 0) {
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            if (DIM == 2 && d == 1) continue;
            double x = (double)c1[d] + f1[d];
            const double L = (double)b.n[d];
            if (x >= L) x -= L;
            if (x < 0.0) x += L;
            if (x >= L) x = 0.0;
            sp.x[d][i] = x;
        }
    } else {
        int cw[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            if (DIM == 2 && d == 1) { cw[d] = 0; continue; }
            cw[d] = wrap_index(c1[d], b.n[d]);
            sp.off[d][i] = f1[d];
        }
        sp.cell[i] = cw[0] + b.n[0] * (cw[1] + b.n[1] * cw[2]);
    }
}

// ------------------------------------------------------------ direct

template <class P, int MODE>
__global__ void __launch_bounds__(256) k_direct(KParams prm, int s) {
    const DevSpecies &sp = prm.species[s];
    const DevBox &b = prm.boxes[sp.box];
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= sp.np) return;
    using FL = LdsField<typename P::FieldT>;
    using JL = LdsJ<typename P::Acc>;
    if (b.dim == 3)
        particle<3, P, MODE, false, FL, JL>(b, sp, i, prm.f, nullptr, nullptr, nullptr, prm.err, nullptr);
    else
        particle<2, P, MODE, false, FL, JL>(b, sp, i, prm.f, nullptr, nullptr, nullptr, prm.err, nullptr);
}

// Particles the tiled kernels found outside their tile plus margin: the
// global-memory update, over every species' straggler list.
template <class P, int MODE>
__global__ void __launch_bounds__(256) k_strag(KParams prm) {
    using FL = LdsField<typename P::FieldT>;
    using JL = LdsJ<typename P::Acc>;
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (int s = 0; s < prm.nsp; ++s) {
        const DevSpecies sp = uniform_species(prm.species[s]);
        const DevBox b = uniform_copy(prm.boxes[sp.box]);
        const long long n = prm.strag_count[s];
        for (long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += stride) {
            const long long i = sp.strag[k];
            if (b.dim == 3)
                particle<3, P, MODE, false, FL, JL>(b, sp, i, prm.f, nullptr, nullptr, nullptr, prm.err, nullptr);
            else
                particle<2, P, MODE, false, FL, JL>(b, sp, i, prm.f, nullptr, nullptr, nullptr, prm.err, nullptr);
        }
    }
}

// ------------------------------------------------------------ tiled / batched

__device__ inline int item_box(const KParams &prm, const Item &it) {
    return it.s >= 0 ? prm.species[it.s].box : -1 - it.s;
}

// Walks the flattened (component, k, j, i) index of an LDS region, i
// fastest, from `start` in steps of `stride`, with the coordinates updated
// by carries instead of a division per element.
struct RegionWalk {
    int i, j, k, c;
    int si, sj, sk, sc;
    int L0, L1, L2;
    __device__ RegionWalk(int start, int stride, int l0, int l1, int l2)
        : L0(l0), L1(l1), L2(l2) {
        decompose(start, i, j, k, c);
        decompose(stride, si, sj, sk, sc);
    }
    __device__ void decompose(int x, int &a, int &b_, int &d, int &e) const {
        a = x % L0; x /= L0;
        b_ = x % L1; x /= L1;
        d = x % L2; e = x / L2;
    }
    __device__ inline void next() {
        i += si; int ci = i >= L0; i -= ci ? L0 : 0;
        j += sj + ci; int cj = j >= L1; j -= cj ? L1 : 0;
        k += sk + cj; int ck = k >= L2; k -= ck ? L2 : 0;
        c += sc + ck;
    }
};

// The particles [p0, p1) of species s in the current tile: lane -> particle
// map: slot k takes particle (k mod G) * S + k / G of the range (S = lane
// stride, G = ceil(n / S)), so that with S equal to the particles per cell
// the lanes of one wave sit in distinct cells and their LDS atomics do not
// collide on one address.  S = 1 is the identity.
template <int DIM, class P, int MODE, bool QUAD>
__device__ __forceinline__ void process_range(const KParams &prm, const DevBox &b, int s, int p0,
                                              int p1, const Tile &tile,
                                              const LdsField<typename P::FieldT> &lf,
                                              const LdsJ<typename P::Acc> &lj) {
    const DevSpecies sp = uniform_species(prm.species[s]);
    // lane_swz: hardware lane bits 4 and 5 trade places (a bijection on each
    // wave's 64 slots; the block is a multiple of 64)
    const int hw = threadIdx.x;
    const int tid = prm.lane_swz ? hw ^ ((((hw >> 4) ^ (hw >> 5)) & 1) * 48) : hw;
    const int bs = blockDim.x;
    const int n = p1 - p0;
    if (n <= 0) return;
    const int S = prm.lane_stride > 1 ? prm.lane_stride : 1;
    const int G = (n + S - 1) / S;
    const int total = G * S;
    int q = tid / G, r = tid - (tid / G) * G;
    const int dq = bs / G, dr = bs - (bs / G) * G;
    if constexpr (MODE == MODE_FUSED) {
        if (QUAD && sp.spread) {
            // Quad slot qs of the range takes quad (qs mod 16) * C + qs / 16
            // (C = ceil(nquads / 16)): the 16 quads of a wave lie C quads
            // apart, so cells holding several whole quads do not fill a
            // wave with one cell's stencil.
            const int C = (((n + 3) >> 2) + 15) >> 4;
            const int tot = C * 64;
            const int rounds = (tot + bs - 1) / bs;
            for (int rd = 0; rd < rounds; ++rd) {
                const int sl = tid + rd * bs;
                const int qs = sl >> 2;
                const int idx = (((qs & 15) * C + (qs >> 4)) << 2) + (sl & 3);
                const bool have = sl < tot && idx < n;
                if (wave_any(have))
                    particle_converged<DIM, P, QUAD>(b, sp, (long long)(p0 + (have ? idx : 0)),
                                                     have, tile, lf, lj, prm.err,
                                                     prm.strag_count + s);
            }
            return;
        }
        // every lane of a wave runs the same slots (the converged path); a
        // wave without a particle in a round (the last, partial round of a
        // range) skips it
        const int rounds = (total + bs - 1) / bs;
        for (int rd = 0; rd < rounds; ++rd) {
            const int sl = tid + rd * bs;
            const int idx = r * S + q;
            const bool have = sl < total && idx < n;
            if (wave_any(have))
                particle_converged<DIM, P, QUAD>(b, sp, (long long)(p0 + (have ? idx : 0)), have,
                                                 tile, lf, lj, prm.err, prm.strag_count + s);
            r += dr;
            q += dq;
            if (r >= G) { r -= G; q += 1; }
        }
    } else {
        for (int sl = tid; sl < total; sl += bs) {
            const int idx = r * S + q;
            if (idx < n)
                particle<DIM, P, MODE, true>(b, sp, (long long)(p0 + idx), prm.f, &tile, &lf, &lj,
                                             prm.err, prm.strag_count + s);
            r += dr;
            q += dq;
            if (r >= G) { r -= G; q += 1; }
        }
    }
}

template <int DIM, class P, int MODE, bool QUAD>
__device__ __forceinline__ void process_item(const KParams &prm, const Item &it, char *smem,
                                             float *red) {
    using FT = typename P::FieldT;
    using A = typename P::Acc;
    const int box = item_box(prm, it);
    const DevBox b = uniform_copy(prm.boxes[box]);
    Tile tile;
    {
        int t = it.t;
        int tx = t % b.nt[0];
        int ty = (t / b.nt[0]) % b.nt[1];
        int tz = t / (b.nt[0] * b.nt[1]);
        int tc[3] = {tx, ty, tz};
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            tile.t0[d] = tc[d] * b.tile[d];
            tile.te[d] = min(b.tile[d], b.n[d] - tile.t0[d]);
        }
    }
    const bool any = b.small != 0;
    LdsField<FT> lf;
    LdsJ<A> lj;
    // field region: cells [t0 - GL, t0 + te + GH) per active axis
    lf.base = (const FT *)smem;
    int JL[3], JW[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        tile.mg[d] = prm.margin[d];
        JL[d] = H::JL + tile.mg[d];
        JW[d] = H::JL + H::JH + 2 * tile.mg[d];
    }
    // Field components: nodes [t0 - lo - mg, t0 + te + hi + mg) per active
    // axis, lo/hi by the component's stagger.  Rows padded to prm.frow
    // (only the first W[c] entries of a row are staged).
    int W[6], FL1[6], FL2[6];
    {
        int acc = 0;
#pragma unroll
        for (int c = 0; c < 6; ++c) {
            int lo[3], w[3];
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                const int st = comp_stagger(c, d);
                lo[d] = gather_lo(O, st) + tile.mg[d];
                w[d] = tile.te[d] + gather_lo(O, st) + gather_hi(O, st) + 2 * tile.mg[d];
            }
            W[c] = w[0];
            lf.o0[c] = tile.t0[0] - lo[0];
            if (prm.falign) {
                // rows from and to multiples of 16 bytes (4 FP32 or 2 FP64
                // nodes: 16-byte copies)
                constexpr int AL = 16 / (int)sizeof(FT);
                const int a0 = lf.o0[c] & ~(AL - 1);
                W[c] = ((lf.o0[c] + w[0] + AL - 1) & ~(AL - 1)) - a0;
                lf.o0[c] = a0;
            }
            lf.L0[c] = max(W[c], prm.frow);
            lf.o2[c] = tile.t0[2] - lo[2];
            FL2[c] = w[2];
            if (DIM == 3) { lf.o1[c] = tile.t0[1] - lo[1]; FL1[c] = w[1]; }
            else { lf.o1[c] = 0; FL1[c] = 1; }
            lf.L01[c] = lf.L0[c] * FL1[c];
            lf.off[c] = acc;
            acc += lf.L01[c] * FL2[c];
        }
    }
    // current region: nodes [t0 - JL, t0 + te + JH) per active axis
    lj.base = (A *)(smem + prm.lds_field_bytes);
    // Row length of the LDS current tile: padded (prm.jrow, from the host)
    // so that a wave's lanes on an 8-wide block of rows hit distinct banks.
    lj.o0 = tile.t0[0] - JL[0]; lj.M0 = max(tile.te[0] + JW[0], prm.jrow);
    lj.o2 = tile.t0[2] - JL[2];
    int M2 = tile.te[2] + JW[2];
    if (DIM == 3) { lj.o1 = tile.t0[1] - JL[1]; lj.M1 = tile.te[1] + JW[1]; }
    else { lj.o1 = 0; lj.M1 = 1; }
    lj.M012 = lj.M0 * lj.M1 * M2;
    lj.N = 3 * lj.M012 - lj.M0 * lj.M1;

    const int tid = threadIdx.x, bs = blockDim.x;
    if (MODE & MODE_PUSH) {
        // Field stage by global -> LDS loads (global_load_lds, into a wave's
        // consecutive LDS words at a wave-uniform base held in M0, which on
        // gfx950 reaches the whole LDS, past 64 KB too): no value passes
        // through a register, so a thread's loads all stay in flight until
        // the wait before the barrier below.  Rows aligned to 16 bytes that
        // need no wrap along x take 16 bytes a lane (4 FP32 or 2 FP64
        // nodes); other FP32 rows one dword a lane; other FP64 rows go
        // through registers, STAGE_BATCH 8-byte loads in flight per thread
        // (faster for FP64 than two dword copies per value).
        const int lane = tid & 63;
        constexpr int AL = 16 / (int)sizeof(FT);
#pragma unroll
        for (int c = 0; c < 6; ++c) {
            const FT *srcf = (const FT *)(c < 3 ? prm.f.E[c] : prm.f.B[c - 3]);
            // 16 bytes a lane: aligned, unpadded rows that need no wrap
            // along x, from a 16-byte aligned array and first cell
            const bool x4 = prm.falign && lf.L0[c] == W[c] && lf.o0[c] >= 0 &&
                            lf.o0[c] + W[c] <= b.n[0] && (b.n[0] & (AL - 1)) == 0 &&
                            (b.cell_base & (AL - 1)) == 0 && ((unsigned long long)srcf & 15) == 0;
            if (x4) {
                unsigned *dst = (unsigned *)((FT *)smem + lf.off[c]);
                const int q = W[c] / AL;    // 16-byte chunks per row
                const int nq = q * FL1[c] * FL2[c];
                RegionWalk w(tid, bs, q, FL1[c], FL2[c]);
                for (int id = tid; id < nq; id += bs, w.next()) {
                    int gj = lf.o1[c] + w.j, gk = lf.o2[c] + w.k;
                    if (any) { gj = wrap_index_any(gj, b.n[1]); gk = wrap_index_any(gk, b.n[2]); }
                    else { gj = wrap_index(gj, b.n[1]); gk = wrap_index(gk, b.n[2]); }
                    const long long e = b.cell_base + lf.o0[c] + AL * w.i +
                                        (long long)b.n[0] * (gj + (long long)b.n[1] * gk);
                    __builtin_amdgcn_global_load_lds((const unsigned *)(srcf + e), dst + 4 * (id - lane),
                                                     16, 0, 0);
                }
            } else if constexpr (sizeof(FT) == 4) {
                unsigned *dst = (unsigned *)((FT *)smem + lf.off[c]);
                const unsigned *src = (const unsigned *)srcf;
                const int nd = lf.L01[c] * FL2[c];
                RegionWalk w(tid, bs, lf.L0[c], FL1[c], FL2[c]);
                for (int id = tid; id < nd; id += bs, w.next()) {
                    if (w.i >= W[c]) continue;
                    int gi = lf.o0[c] + w.i, gj = lf.o1[c] + w.j, gk = lf.o2[c] + w.k;
                    if (any) { gi = wrap_index_any(gi, b.n[0]); gj = wrap_index_any(gj, b.n[1]); gk = wrap_index_any(gk, b.n[2]); }
                    else { gi = wrap_index(gi, b.n[0]); gj = wrap_index(gj, b.n[1]); gk = wrap_index(gk, b.n[2]); }
                    const long long e = b.cell_base + gi + (long long)b.n[0] * (gj + (long long)b.n[1] * gk);
                    __builtin_amdgcn_global_load_lds(src + e, dst + (id - lane), 4, 0, 0);
                }
            } else {
                // through registers: STAGE_BATCH loads in flight per thread
                // before their LDS stores (one at a time, each store waits
                // for its load's full latency)
                FT *dst = (FT *)smem + lf.off[c];
                const int n = lf.L01[c] * FL2[c];
                RegionWalk w(tid, bs, lf.L0[c], FL1[c], FL2[c]);
                for (int idx0 = tid; idx0 < n; idx0 += STAGE_BATCH * bs) {
                    const FT *src[STAGE_BATCH];
                    bool ok[STAGE_BATCH];
#pragma unroll
                    for (int u = 0; u < STAGE_BATCH; ++u) {
                        // addresses first (only those of staged entries are read)
                        ok[u] = idx0 + u * bs < n && w.i < W[c];
                        int gi = lf.o0[c] + w.i, gj = lf.o1[c] + w.j, gk = lf.o2[c] + w.k;
                        if (any) { gi = wrap_index_any(gi, b.n[0]); gj = wrap_index_any(gj, b.n[1]); gk = wrap_index_any(gk, b.n[2]); }
                        else { gi = wrap_index(gi, b.n[0]); gj = wrap_index(gj, b.n[1]); gk = wrap_index(gk, b.n[2]); }
                        src[u] = srcf + b.cell_base + gi + (long long)b.n[0] * (gj + (long long)b.n[1] * gk);
                        w.next();
                    }
                    FT v[STAGE_BATCH];
#pragma unroll
                    for (int u = 0; u < STAGE_BATCH; ++u) v[u] = ok[u] ? *src[u] : FT(0);
#pragma unroll
                    for (int u = 0; u < STAGE_BATCH; ++u)
                        if (ok[u]) dst[idx0 + u * bs] = v[u];
                }
            }
        }
    }
    if (MODE & MODE_DEPOSIT) {
        const int n = lj.N;
        for (int idx = tid; idx < n; idx += bs) lj.base[idx] = A(0);
    }
    constexpr bool FIXED = LdsJ<A>::FIXED && (MODE & MODE_DEPOSIT);
    if constexpr (FIXED) {
        // Scale of the fixed-point current tile: the largest |charge factor|
        // (q w dx_d / (dt dV), and q w / dV for the 2D out-of-plane current)
        // over the item's particles, rounded up to a power of two, maps to
        // 2^30.  A contribution is that factor times a prefix sum of shape
        // differences and a line weight, both at most 1 in magnitude, so it
        // stays below 2^31 as an integer.  Non-finite weights set the range
        // flag.
        float m = 0.0f;
        bool bad = false;
        auto scan = [&](int s, int p0, int p1) {
            const DevSpecies &sp = prm.species[s];
            const double dV = b.dx[0] * b.dx[1] * b.dx[2];
            double qb = fabs(sp.q) / dV;
#pragma unroll
            for (int d = 0; d < 3; ++d) qb = fmax(qb, fabs(sp.q * b.dx[d] / (b.dt * dV)));
            const float Q = (float)qb;
            const float *w = (const float *)sp.w;
            // four loads in flight per thread
            for (int p = p0 + tid; p < p1; p += 4 * bs) {
                float x[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) x[u] = p + u * bs < p1 ? fabsf(w[p + u * bs]) * Q : 0.0f;
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    bad = bad || !(x[u] <= 3.0e38f);
                    m = fmaxf(m, x[u]);
                }
            }
        };
        if (it.s >= 0) {
            scan(it.s, it.p0, it.p1);
        } else {
            for (int k = prm.box_sp_off[box]; k < prm.box_sp_off[box + 1]; ++k) {
                const int s = prm.box_sp[k];
                const int *off = prm.species[s].tile_off;
                scan(s, off[it.t], off[it.t + 1]);
            }
        }
        if (bad) flag_range(prm.err);
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o));
        if ((tid & 63) == 0) red[tid >> 6] = m;
    }
    // the global -> LDS copies of the field stage have landed
    if (MODE & MODE_PUSH) __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if constexpr (FIXED) {
        float m = 0.0f;
        for (int wv = 0; wv < (bs >> 6); ++wv) m = fmaxf(m, red[wv]);
        int e = 0;
        (void)frexpf(m, &e);              // m < 2^e
        e = max(e, -90);
        lj.scale = ldexpf(1.0f, 30 - e);
        lj.unscale = ldexp(1.0, e - 30);
    } else {
        lj.scale = 1.0f;
        lj.unscale = 1.0;
    }
    if (it.s >= 0) {
        process_range<DIM, P, MODE, QUAD>(prm, b, it.s, it.p0, it.p1, tile, lf, lj);
    } else {
        for (int k = prm.box_sp_off[box]; k < prm.box_sp_off[box + 1]; ++k) {
            const int s = prm.box_sp[k];
            const int *off = prm.species[s].tile_off;
            process_range<DIM, P, MODE, QUAD>(prm, b, s, off[it.t], off[it.t + 1], tile, lf, lj);
        }
    }
    __syncthreads();
    if (MODE & MODE_DEPOSIT) {
        const int n = lj.N;
        // component arrays selected in registers, not indexed in memory
        double *const J0 = prm.f.J[0], *const J1 = prm.f.J[1], *const J2 = prm.f.J[2];
        RegionWalk w(tid, bs, lj.M0, lj.M1, M2);
        for (int idx = tid; idx < n; idx += bs, w.next()) {
            const A v = lj.base[idx];
            if (v == A(0)) continue;
            const double jv = FIXED ? (double)v * lj.unscale : (double)v;
            int gi = lj.o0 + w.i, gj = lj.o1 + w.j, gk = lj.o2 + w.k;
            if (any) { gi = wrap_index_any(gi, b.n[0]); gj = wrap_index_any(gj, b.n[1]); gk = wrap_index_any(gk, b.n[2]); }
            else { gi = wrap_index(gi, b.n[0]); gj = wrap_index(gj, b.n[1]); gk = wrap_index(gk, b.n[2]); }
            double *Jc = w.c == 0 ? J0 : w.c == 1 ? J1 : J2;
            unsafeAtomicAdd(&Jc[b.cell_base + gi + (long long)b.n[0] * (gj + (long long)b.n[1] * gk)], jv);
        }
    }
    __syncthreads();
}

// DIMS: 3 or 2 when every box of the context has that dimensionality (one
// code path, fewer registers), 0 for a mix.
template <class P, int MODE, bool PERSISTENT, int DIMS, bool QUAD>
__global__ void __launch_bounds__(P::MAX_BLOCK) k_tiled(KParams prm) {
    extern __shared__ __attribute__((aligned(16))) char smem[];
    __shared__ Item cur;
    __shared__ float red[P::MAX_BLOCK / 64];
    for (int round = 0;; ++round) {
        Item it;
        if (PERSISTENT) {
            if (threadIdx.x == 0) {
                int idx = atomicAdd(prm.queue, 1);
                cur = idx < *prm.nitems ? prm.items[idx] : Item{0, -1, 0, 0};
            }
            __syncthreads();
            // the item is the same for the whole workgroup
            it.s = __builtin_amdgcn_readfirstlane(cur.s);
            it.t = __builtin_amdgcn_readfirstlane(cur.t);
            it.p0 = __builtin_amdgcn_readfirstlane(cur.p0);
            it.p1 = __builtin_amdgcn_readfirstlane(cur.p1);
            __syncthreads();
            if (it.t < 0) return;
        } else {
            if (round > 0) return;
            const int bidx = blockIdx.x;
            int s = 0;
            while (s + 1 < prm.nsp && prm.sp_tile_prefix[s + 1] <= bidx) ++s;
            const int t = bidx - prm.sp_tile_prefix[s];
            const int *off = prm.species[s].tile_off;
            it = Item{s, t, off[t], off[t + 1]};
        }
        if (it.p1 <= it.p0) continue;
        if constexpr (DIMS == 3) {
            process_item<3, P, MODE, QUAD>(prm, it, smem, red);
        } else if constexpr (DIMS == 2) {
            process_item<2, P, MODE, QUAD>(prm, it, smem, red);
        } else {
            const DevBox &b = prm.boxes[item_box(prm, it)];
            if (b.dim == 3) process_item<3, P, MODE, QUAD>(prm, it, smem, red);
            else process_item<2, P, MODE, QUAD>(prm, it, smem, red);
        }
    }
}

template <class P, int MODE, bool PERS, bool QUAD>
hipError_t launch_tiled_q(const KParams &prm, int dims, int grid, int block, size_t lds,
                          hipStream_t st) {
    if (dims == 3) {
        hipLaunchKernelGGL((k_tiled<P, MODE, PERS, 3, QUAD>), dim3(grid), dim3(block), lds, st, prm);
    } else if (dims == 2) {
        hipLaunchKernelGGL((k_tiled<P, MODE, PERS, 2, QUAD>), dim3(grid), dim3(block), lds, st, prm);
    } else {
        hipLaunchKernelGGL((k_tiled<P, MODE, PERS, 0, QUAD>), dim3(grid), dim3(block), lds, st, prm);
    }
    return hipGetLastError();
}

// Fused kernels: per dimensionality, with quad pooling of the deposit when
// lane stride 1 meets the quads-first order (prm.quad).  Push-only /
// deposit-only kernels: mixed form.
template <class P, int MODE, bool PERS>
hipError_t launch_tiled_dims(const KParams &prm, int dims, int grid, int block, size_t lds,
                             hipStream_t st) {
    if constexpr (MODE == MODE_FUSED) {
        if (prm.quad) return launch_tiled_q<P, MODE, PERS, true>(prm, dims, grid, block, lds, st);
        return launch_tiled_q<P, MODE, PERS, false>(prm, dims, grid, block, lds, st);
    }
    hipLaunchKernelGGL((k_tiled<P, MODE, PERS, 0, false>), dim3(grid), dim3(block), lds, st, prm);
    return hipGetLastError();
}

template <class P, int MODE>
hipError_t launch_mode_other(const KParams &prm, int form, int grid, int block, size_t lds,
                             int species, hipStream_t st) {
    if (form == 0) {
        hipLaunchKernelGGL((k_direct<P, MODE>), dim3(grid), dim3(256), 0, st, prm, species);
        return hipGetLastError();
    }
    if (form == 3) {
        hipLaunchKernelGGL((k_strag<P, MODE>), dim3(grid), dim3(256), 0, st, prm);
        return hipGetLastError();
    }
    if constexpr (MODE == MODE_FUSED) {
        return hipErrorInvalidValue;     // fused tiled kernels live in their own unit
    } else {
        if (form == 1) return launch_tiled_dims<P, MODE, false>(prm, 0, grid, block, lds, st);
        return launch_tiled_dims<P, MODE, true>(prm, 0, grid, block, lds, st);
    }
}

template <class P, int MODE, bool PERS, int DIMS, bool QUAD>
hipError_t set_lds(int bytes) {
    return hipFuncSetAttribute((const void *)&k_tiled<P, MODE, PERS, DIMS, QUAD>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
}

// Charge density on nodes (FP64, a check): rho += q w S S S / dV.
template <class P>
__global__ void k_rho(KParams prm, int s, double *rho) {
    const DevSpecies &sp = prm.species[s];
    const DevBox &b = prm.boxes[sp.box];
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= sp.np) return;
    int c[3];
    double f[3];
    bool ok;
    if constexpr (P::PREC == 0) {
        ok = P::load(b, sp.x, i, c, f);
    } else {
        float ff[3];
        ok = P::load(b, sp.cell, sp.off, i, c, ff);
#pragma unroll
        for (int d = 0; d < 3; ++d) f[d] = (double)ff[d];
    }
    if (!ok) { flag_range(prm.err); return; }
    GWin<O, double> g[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        if (b.dim == 2 && d == 1) {
            g[d].base = 0;
            for (int m = 0; m <= O; ++m) g[d].w[m] = (m == 0) ? 1.0 : 0.0;
            continue;
        }
        g[d] = gather_window<O, double>(c[d], f[d], 0);
    }
    const double qw = sp.q * ((const typename P::R *)sp.w)[i] / (b.dx[0] * b.dx[1] * b.dx[2]);
    const int ny = (b.dim == 2) ? 1 : O + 1;
    for (int kk = 0; kk <= O; ++kk)
        for (int jj = 0; jj < ny; ++jj)
            for (int ii = 0; ii <= O; ++ii) {
                double v = qw * g[0].w[ii] * g[1].w[jj] * g[2].w[kk];
                if (v == 0.0) continue;
                int a = wrap_index_any(g[0].base + ii, b.n[0]);
                int bb = wrap_index_any(g[1].base + jj, b.n[1]);
                int cc = wrap_index_any(g[2].base + kk, b.n[2]);
                unsafeAtomicAdd(&rho[a + (long long)b.n[0] * (bb + (long long)b.n[1] * cc)], v);
            }
}

}  // namespace

#define PIC_CAT2(a, b) a##b
#define PIC_CAT(a, b) PIC_CAT2(a, b)
#define PIC_NAME(f) PIC_CAT(PIC_CAT(PIC_CAT(f##_o, PIC_ORDER), PIC_CAT(_p, PIC_PREC)), PIC_CAT(_t, PIC_PART))

using PP = typename std::conditional<PIC_PREC == 0, F64, Split>::type;

#if PIC_PART == 0
// direct and straggler kernels (every mode), push-only / deposit-only tiled
// kernels, and the charge-density check
hipError_t PIC_NAME(launch_particles)(const KParams &prm, int form, int mode, int dims, int grid,
                                      int block, size_t lds, int species, hipStream_t st) {
    (void)dims;
    if (mode == MODE_PUSH) return launch_mode_other<PP, MODE_PUSH>(prm, form, grid, block, lds, species, st);
    if (mode == MODE_DEPOSIT) return launch_mode_other<PP, MODE_DEPOSIT>(prm, form, grid, block, lds, species, st);
    return launch_mode_other<PP, MODE_FUSED>(prm, form, grid, block, lds, species, st);
}

hipError_t PIC_NAME(particles_lds_limit)(int bytes) {
    hipError_t e = hipSuccess;
    if (e == hipSuccess) e = set_lds<PP, MODE_PUSH, false, 0, false>(bytes);
    if (e == hipSuccess) e = set_lds<PP, MODE_PUSH, true, 0, false>(bytes);
    if (e == hipSuccess) e = set_lds<PP, MODE_DEPOSIT, false, 0, false>(bytes);
    if (e == hipSuccess) e = set_lds<PP, MODE_DEPOSIT, true, 0, false>(bytes);
    return e;
}

hipError_t PIC_NAME(launch_rho)(const KParams &prm, int species, long long np, double *rho,
                                hipStream_t st) {
    if (np == 0) return hipSuccess;
    dim3 g((unsigned)((np + 255) / 256)), bl(256);
    hipLaunchKernelGGL(k_rho<PP>, g, bl, 0, st, prm, species, rho);
    return hipGetLastError();
}
#else
// fused tiled kernels: PIC_PART 1 the one-workgroup-per-tile form, 2 the
// persistent (batched) form
constexpr bool PERS_PART = PIC_PART == 2;

hipError_t PIC_NAME(launch_particles)(const KParams &prm, int form, int mode, int dims, int grid,
                                      int block, size_t lds, int species, hipStream_t st) {
    (void)species;
    if (mode != MODE_FUSED || form != (PERS_PART ? 2 : 1)) return hipErrorInvalidValue;
    return launch_tiled_dims<PP, MODE_FUSED, PERS_PART>(prm, dims, grid, block, lds, st);
}

hipError_t PIC_NAME(particles_lds_limit)(int bytes) {
    hipError_t e = hipSuccess;
    if (e == hipSuccess) e = set_lds<PP, MODE_FUSED, PERS_PART, 0, false>(bytes);
    if (e == hipSuccess) e = set_lds<PP, MODE_FUSED, PERS_PART, 2, false>(bytes);
    if (e == hipSuccess) e = set_lds<PP, MODE_FUSED, PERS_PART, 3, false>(bytes);
    if (e == hipSuccess) e = set_lds<PP, MODE_FUSED, PERS_PART, 0, true>(bytes);
    if (e == hipSuccess) e = set_lds<PP, MODE_FUSED, PERS_PART, 2, true>(bytes);
    if (e == hipSuccess) e = set_lds<PP, MODE_FUSED, PERS_PART, 3, true>(bytes);
    return e;
}
#endif

}  // namespace pic
