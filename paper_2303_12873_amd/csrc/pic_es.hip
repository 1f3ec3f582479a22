// Electrostatic variant of the step (the paper's codes include an
// electrostatic solver beside the electromagnetic one, Sec. IV): the charge
// density is deposited (pic_deposit_rho), its mean removed (a neutralising
// background), the discrete periodic Poisson equation -div grad phi = rho
// solved by conjugate gradients with the 7-point Yee Laplacian (5 points in
// 2D), and E = -grad phi formed at the Yee E points, so that div E = rho
// holds to the solver's tolerance.  The particles then gather E (the same
// shape factors as the EM step), take the Boris step with B = 0 (an
// electric kick), advance and wrap; no current is deposited.
#include <algorithm>
#include <type_traits>

#include "pic_dev.h"
#include "pic_math.h"
#include "pic_aux.h"

namespace pic {
namespace {

inline unsigned nblocks(long long n, int bs) { return (unsigned)((n + bs - 1) / bs); }

struct Ijk {
    int i, j, k;
};

__device__ inline Ijk decompose(const DevBox &b, long long c) {
    Ijk r;
    r.i = (int)(c % b.n[0]);
    const long long t = c / b.n[0];
    r.j = (int)(t % b.n[1]);
    r.k = (int)(t / b.n[1]);
    return r;
}

__device__ inline long long at(const DevBox &b, int i, int j, int k) {
    i = wrap_index_any(i, b.n[0]);
    j = wrap_index_any(j, b.n[1]);
    k = wrap_index_any(k, b.n[2]);
    return i + (long long)b.n[0] * (j + (long long)b.n[1] * k);
}

// y = -div grad x (periodic, Yee differences) over box-local arrays.
__global__ void k_neg_lap(const DevBox *boxes, int bi, const double *x, double *y) {
    const DevBox &b = boxes[bi];
    long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= b.ncells) return;
    const Ijk p = decompose(b, c);
    const double xc = x[c];
    const double ix2 = 1.0 / (b.dx[0] * b.dx[0]), iz2 = 1.0 / (b.dx[2] * b.dx[2]);
    double v = (2.0 * xc - x[at(b, p.i + 1, p.j, p.k)] - x[at(b, p.i - 1, p.j, p.k)]) * ix2 +
               (2.0 * xc - x[at(b, p.i, p.j, p.k + 1)] - x[at(b, p.i, p.j, p.k - 1)]) * iz2;
    if (b.dim == 3) {
        const double iy2 = 1.0 / (b.dx[1] * b.dx[1]);
        v += (2.0 * xc - x[at(b, p.i, p.j + 1, p.k)] - x[at(b, p.i, p.j - 1, p.k)]) * iy2;
    }
    y[c] = v;
}

__device__ inline double block_sum(double v, double *red) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    if (l == 0) red[w] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0)
        for (int k = 0; k < (int)(blockDim.x >> 6); ++k) t += red[k];
    __syncthreads();
    return t;
}

// part[block] = sum of a[i] * b[i] over the block's grid-stride share.
__global__ void __launch_bounds__(256) k_dot(const double *a, const double *b, long long n,
                                             double *part) {
    __shared__ double red[4];
    double s = 0.0;
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        s += a[i] * b[i];
    s = block_sum(s, red);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// out = sum of part[0 .. np) in order (one thread: fixed order).
__global__ void k_sum_parts(const double *part, int np, double *out) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double s = 0.0;
    for (int i = 0; i < np; ++i) s += part[i];
    *out = s;
}

// x -= mean(x) (the mean from sc[0] = sum x, divided by n).
__global__ void k_remove_mean(double *x, long long n, const double *sum) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] -= *sum / (double)n;
}

// CG scalars: sc[0] = r.r, sc[1] = p.Ap, sc[2] = r_new.r_new.
// alpha = r.r / p.Ap: x += alpha p, r -= alpha Ap.
__global__ void k_cg_xr(double *x, double *r, const double *p, const double *ap, long long n,
                        const double *sc) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double alpha = sc[1] != 0.0 ? sc[0] / sc[1] : 0.0;
    x[i] += alpha * p[i];
    r[i] -= alpha * ap[i];
}

// beta = r_new.r_new / r.r: p = r + beta p; then r.r <- r_new.r_new.
__global__ void k_cg_p(double *p, const double *r, long long n, const double *sc) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double beta = sc[0] != 0.0 ? sc[2] / sc[0] : 0.0;
    p[i] = r[i] + beta * p[i];
}

__global__ void k_copy_scalar(double *sc, int to, int from) { sc[to] = sc[from]; }

__global__ void k_copy_d(const double *a, double *b, long long n) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = a[i];
}

__global__ void k_zero_d(double *a, long long n) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] = 0.0;
}

// E = -grad phi at the Yee E points of box bi (E in the context's precision).
template <typename T>
__global__ void k_es_field(const DevBox *boxes, int bi, const double *phi, DevFields f) {
    const DevBox &b = boxes[bi];
    long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= b.ncells) return;
    const Ijk p = decompose(b, c);
    const double pc = phi[c];
    T *Ex = (T *)f.E[0] + b.cell_base, *Ey = (T *)f.E[1] + b.cell_base, *Ez = (T *)f.E[2] + b.cell_base;
    Ex[c] = (T)(-(phi[at(b, p.i + 1, p.j, p.k)] - pc) / b.dx[0]);
    Ey[c] = b.dim == 3 ? (T)(-(phi[at(b, p.i, p.j + 1, p.k)] - pc) / b.dx[1]) : T(0);
    Ez[c] = (T)(-(phi[at(b, p.i, p.j, p.k + 1)] - pc) / b.dx[2]);
}

// ------------------------------------------------------------ push in E

template <int O, typename R, typename FT>
__device__ R gather_comp(const DevBox &b, const FT *F, const GWin<O, R> &wx, const GWin<O, R> &wy,
                         const GWin<O, R> &wz) {
    R s = R(0);
    const int ny = b.dim == 3 ? O : 0;
    for (int kk = 0; kk <= O; ++kk)
        for (int jj = 0; jj <= ny; ++jj) {
            R sx = R(0);
            for (int ii = 0; ii <= O; ++ii)
                sx += wx.w[ii] * (R)F[at(b, wx.base + ii, b.dim == 3 ? wy.base + jj : 0, wz.base + kk)];
            s += (b.dim == 3 ? wy.w[jj] : R(1)) * wz.w[kk] * sx;
        }
    return s;
}

// One thread per particle of species s: gather E at x^n (each component on
// its own Yee points), u += (q dt / m) E (the Boris step with B = 0),
// advance, wrap.  PREC 0: FP64 positions; 1: int32 cell + FP32 offsets
// (carry as in the EM step).
template <int O, int PREC>
__global__ void k_es_push(const DevSpecies *spt, int s, const DevBox *boxes, DevFields f, int *err) {
    using R = typename std::conditional<PREC == 0, double, float>::type;
    const DevSpecies &sp = spt[s];
    const DevBox &b = boxes[sp.box];
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= sp.np) return;
    int c[3] = {0, 0, 0};
    R fr[3] = {R(0), R(0), R(0)};
    if (PREC == 0) {
        for (int d = 0; d < 3; ++d) {
            if (b.dim == 2 && d == 1) continue;
            const double x = sp.x[d][i];
            if (!(x >= 0.0 && x < (double)b.n[d])) { atomicOr(err, 1); return; }
            const double fl = floor(x);
            c[d] = (int)fl;
            fr[d] = (R)(x - fl);
        }
    } else {
        const int cell = sp.cell[i];
        if (cell < 0 || (long long)cell >= b.ncells) { atomicOr(err, 1); return; }
        c[0] = cell % b.n[0];
        c[1] = (cell / b.n[0]) % b.n[1];
        c[2] = cell / (b.n[0] * b.n[1]);
        for (int d = 0; d < 3; ++d) {
            if (b.dim == 2 && d == 1) continue;
            const float v = sp.off[d][i];
            if (!(v >= 0.0f && v < 1.0f)) { atomicOr(err, 1); return; }
            fr[d] = (R)v;
        }
    }
    GWin<O, R> g0[3], g1[3];
    for (int d = 0; d < 3; ++d) {
        g0[d] = gather_window<O, R>(c[d], fr[d], 0);
        if (sp.galerkin) g1[d] = gather_window_galerkin<O, R>(c[d], fr[d]);
        else g1[d] = gather_window<O, R>(c[d], fr[d], 1);
    }
    using FT = R;
    const FT *Ex = (const FT *)f.E[0] + b.cell_base, *Ey = (const FT *)f.E[1] + b.cell_base,
             *Ez = (const FT *)f.E[2] + b.cell_base;
    R E[3];
    E[0] = gather_comp<O, R>(b, Ex, g1[0], g0[1], g0[2]);
    E[1] = gather_comp<O, R>(b, Ey, g0[0], g1[1], g0[2]);
    E[2] = gather_comp<O, R>(b, Ez, g0[0], g0[1], g1[2]);
    R *u[3] = {(R *)sp.u[0], (R *)sp.u[1], (R *)sp.u[2]};
    const R h = (R)(sp.q * b.dt / (2.0 * sp.m));
    const R zero[3] = {R(0), R(0), R(0)};
    R uu[3] = {u[0][i], u[1][i], u[2][i]};
    push_momentum<R>(sp.pusher, h, E, zero, uu);
    const R gi = R(1) / sqrt(R(1) + uu[0] * uu[0] + uu[1] * uu[1] + uu[2] * uu[2]);
    R disp[3];
    bool good = true;
    for (int d = 0; d < 3; ++d) {
        disp[d] = (b.dim == 2 && d == 1) ? R(0) : (R)b.dt * uu[d] * gi / (R)b.dx[d];
        good = good && fabs(disp[d]) < R(0.999);
    }
    if (!good) { atomicOr(err, 1); return; }
    for (int d = 0; d < 3; ++d) u[d][i] = uu[d];
    if (PREC == 0) {
        for (int d = 0; d < 3; ++d) {
            if (b.dim == 2 && d == 1) continue;
            double x = ((double)c[d] + (double)fr[d]) + (double)disp[d];
            const double L = (double)b.n[d];
            if (x >= L) x -= L;
            if (x < 0.0) x += L;
            if (x >= L) x = 0.0;
            sp.x[d][i] = x;
        }
    } else {
        int cw[3];
        for (int d = 0; d < 3; ++d) {
            if (b.dim == 2 && d == 1) { cw[d] = 0; continue; }
            float fr1 = (float)fr[d] + (float)disp[d];
            int c1 = c[d];
            if (fr1 >= 1.0f) { c1 += 1; fr1 -= 1.0f; }
            else if (fr1 < 0.0f) {
                c1 -= 1; fr1 += 1.0f;
                if (fr1 == 1.0f) { fr1 = 0.0f; c1 += 1; }
            }
            cw[d] = wrap_index(c1, b.n[d]);
            sp.off[d][i] = fr1;
        }
        sp.cell[i] = cw[0] + b.n[0] * (cw[1] + b.n[1] * cw[2]);
    }
}

}  // namespace

hipError_t launch_neg_lap(const DevBox *boxes, int bi, long long n, const double *x, double *y,
                          hipStream_t st) {
    hipLaunchKernelGGL(k_neg_lap, dim3(nblocks(n, 256)), dim3(256), 0, st, boxes, bi, x, y);
    return hipGetLastError();
}

// out = a . b (deterministic two-pass sum); part: ES_DOT_GRID doubles.
hipError_t launch_dot(const double *a, const double *b, long long n, double *part, double *out,
                      hipStream_t st) {
    const unsigned g = std::max(1u, std::min(nblocks(n, 256), (unsigned)ES_DOT_GRID));
    hipLaunchKernelGGL(k_dot, dim3(g), dim3(256), 0, st, a, b, n, part);
    hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(64), 0, st, (const double *)part, (int)g, out);
    return hipGetLastError();
}

hipError_t launch_remove_mean(double *x, long long n, double *part, double *sc, const double *ones,
                              hipStream_t st) {
    hipError_t e = launch_dot(x, ones, n, part, sc, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_remove_mean, dim3(nblocks(n, 256)), dim3(256), 0, st, x, n, (const double *)sc);
    return hipGetLastError();
}

hipError_t launch_cg_xr(double *x, double *r, const double *p, const double *ap, long long n,
                        const double *sc, hipStream_t st) {
    hipLaunchKernelGGL(k_cg_xr, dim3(nblocks(n, 256)), dim3(256), 0, st, x, r, p, ap, n, sc);
    return hipGetLastError();
}

hipError_t launch_cg_p(double *p, const double *r, long long n, const double *sc, hipStream_t st) {
    hipLaunchKernelGGL(k_cg_p, dim3(nblocks(n, 256)), dim3(256), 0, st, p, r, n, sc);
    return hipGetLastError();
}

hipError_t launch_copy_scalar(double *sc, int to, int from, hipStream_t st) {
    hipLaunchKernelGGL(k_copy_scalar, dim3(1), dim3(1), 0, st, sc, to, from);
    return hipGetLastError();
}

hipError_t launch_copy_d(const double *a, double *b, long long n, hipStream_t st) {
    hipLaunchKernelGGL(k_copy_d, dim3(nblocks(n, 256)), dim3(256), 0, st, a, b, n);
    return hipGetLastError();
}

hipError_t launch_zero_d(double *a, long long n, hipStream_t st) {
    hipLaunchKernelGGL(k_zero_d, dim3(nblocks(n, 256)), dim3(256), 0, st, a, n);
    return hipGetLastError();
}

hipError_t launch_es_field(int prec, const DevBox *boxes, int bi, long long n, const double *phi,
                           const DevFields &f, hipStream_t st) {
    if (prec == 0)
        hipLaunchKernelGGL(k_es_field<double>, dim3(nblocks(n, 256)), dim3(256), 0, st, boxes, bi, phi, f);
    else
        hipLaunchKernelGGL(k_es_field<float>, dim3(nblocks(n, 256)), dim3(256), 0, st, boxes, bi, phi, f);
    return hipGetLastError();
}

hipError_t launch_es_push(int order, int prec, const DevSpecies *spt, int s, long long np,
                          const DevBox *boxes, const DevFields &f, int *err, hipStream_t st) {
    if (np == 0) return hipSuccess;
    const dim3 g(nblocks(np, 256)), bl(256);
#define PIC_ES(OO, PP) hipLaunchKernelGGL((k_es_push<OO, PP>), g, bl, 0, st, spt, s, boxes, f, err)
    if (prec == 0) {
        if (order == 1) PIC_ES(1, 0); else if (order == 2) PIC_ES(2, 0); else PIC_ES(3, 0);
    } else {
        if (order == 1) PIC_ES(1, 1); else if (order == 2) PIC_ES(2, 1); else PIC_ES(3, 1);
    }
#undef PIC_ES
    return hipGetLastError();
}

}  // namespace pic
