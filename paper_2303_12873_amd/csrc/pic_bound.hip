// The laser-plasma boundaries around the periodic step: a laser antenna
// (current sheet), and a moving window along z kept as a circular offset of
// the z index (no field data moves): advancing the window zeroes the array
// layer that leaves the frame's bottom and becomes its new top, removes the
// particles in it, appends the caller's injected particles and advances the
// offset.  The absorbing layers that bound z live in the Yee kernels
// (pic_aux.hip), at the window-frame ends.
#include <algorithm>

#include "pic_dev.h"
#include "pic_aux.h"

namespace pic {
namespace {

inline unsigned nblocks(long long n, int bs) { return (unsigned)((n + bs - 1) / bs); }

// Current sheet in cell layer (k_w + zoff) mod n_z at the E_x points:
// J_x += -2 E0 exp(-r^2/w^2) exp(-((t - t0)/tau)^2) sin(omega (t - t0)) / dz.
__global__ void k_antenna(double *Jx, const DevBox *boxes, int bi, AntennaArgs an, double t) {
    const DevBox &b = boxes[bi];
    const long long nxy = (long long)b.n[0] * b.n[1];
    long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nxy) return;
    const int i = (int)(c % b.n[0]), j = (int)(c / b.n[0]);
    int k = (an.k + b.zoff) % b.n[2];
    if (k < 0) k += b.n[2];
    const double s = (t - an.t0) / an.tau;
    const double amp = -2.0 * an.E0 * exp(-s * s) * sin(an.omega * (t - an.t0)) / b.dx[2];
    const double x = (i + 0.5) * b.dx[0] - an.x0;
    const double y = b.dim == 3 ? (double)j * b.dx[1] - an.y0 : 0.0;
    Jx[b.cell_base + c + nxy * k] += amp * exp(-(x * x + y * y) / (an.waist * an.waist));
}

// E and B of array layer k set to zero.
template <typename T>
__global__ void k_zero_layer(SlabComps<T> f, const DevBox *boxes, int bi, int k) {
    const DevBox &b = boxes[bi];
    const long long nxy = (long long)b.n[0] * b.n[1];
    long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nxy) return;
    const long long g = b.cell_base + c + nxy * k;
    for (int q = 0; q < 6; ++q) f.c[q][g] = T(0);
}

__global__ void k_box_zoff(DevBox *boxes, int bi, int zoff) { boxes[bi].zoff = zoff; }

// Particles that stay: not in array layer k.
template <int PREC>
__global__ void k_win_flags(MigSpecies m, int k, int nxy, int *stay) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m.np) return;
    int z;
    if (PREC == 0) z = (int)floor(((const double *)m.a[m.zi])[i]);
    else z = ((const int *)m.a[0])[i] / nxy;
    stay[i] = z != k;
}

template <typename E>
__global__ void k_win_compact(MigSpecies m, const int *stay, const int *pos, MigBuffers sb) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m.np || !stay[i]) return;
    const long long k = pos[i];
    for (int a = 0; a < m.na; ++a) ((E *)sb.stay[a])[k] = ((const E *)m.a[a])[i];
}

// Species arrays <- the nstay stayers, then the nin injected particles with
// their window-frame z moved to the array frame (+ zoff mod n_z).
template <typename E, int PREC>
__global__ void k_win_fill(MigSpecies m, long long nstay, MigBuffers sb, MigSpecies in,
                           int zoff, int nz, int nxy) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nstay + in.np) return;
    for (int a = 0; a < m.na; ++a) {
        E v;
        if (i < nstay) {
            v = ((const E *)sb.stay[a])[i];
        } else {
            v = ((const E *)in.a[a])[i - nstay];
            if (PREC == 0 && a == m.zi) {
                double z = (double)v + (double)zoff;
                z -= (double)nz * floor(z / (double)nz);
                v = (E)z;
            }
            if (PREC == 1 && a == 0) {
                const int cell = (int)v;
                int kz = cell / nxy + zoff;
                kz %= nz;
                if (kz < 0) kz += nz;
                v = (E)(cell % nxy + nxy * kz);
            }
        }
        ((E *)m.a[a])[i] = v;
    }
}

}  // namespace

hipError_t launch_antenna(double *Jx, const DevBox *boxes, int bi, long long nxy,
                          const AntennaArgs &an, double t, hipStream_t st) {
    if (nxy == 0) return hipSuccess;
    hipLaunchKernelGGL(k_antenna, dim3(nblocks(nxy, 256)), dim3(256), 0, st, Jx, boxes, bi, an, t);
    return hipGetLastError();
}

hipError_t launch_zero_layer(int prec, void *const *comps, const DevBox *boxes, int bi, long long nxy,
                             int k, hipStream_t st) {
    if (nxy == 0) return hipSuccess;
    if (prec == 0) {
        SlabComps<double> f;
        for (int q = 0; q < 6; ++q) f.c[q] = (double *)comps[q];
        hipLaunchKernelGGL(k_zero_layer<double>, dim3(nblocks(nxy, 256)), dim3(256), 0, st, f,
                           boxes, bi, k);
    } else {
        SlabComps<float> f;
        for (int q = 0; q < 6; ++q) f.c[q] = (float *)comps[q];
        hipLaunchKernelGGL(k_zero_layer<float>, dim3(nblocks(nxy, 256)), dim3(256), 0, st, f,
                           boxes, bi, k);
    }
    return hipGetLastError();
}

hipError_t launch_box_zoff(DevBox *boxes, int bi, int zoff, hipStream_t st) {
    hipLaunchKernelGGL(k_box_zoff, dim3(1), dim3(1), 0, st, boxes, bi, zoff);
    return hipGetLastError();
}

hipError_t launch_win_flags(int prec, const MigSpecies &m, int k, int nxy, int *stay,
                            hipStream_t st) {
    if (m.np == 0) return hipSuccess;
    if (prec == 0)
        hipLaunchKernelGGL(k_win_flags<0>, dim3(nblocks(m.np, 256)), dim3(256), 0, st, m, k, nxy, stay);
    else
        hipLaunchKernelGGL(k_win_flags<1>, dim3(nblocks(m.np, 256)), dim3(256), 0, st, m, k, nxy, stay);
    return hipGetLastError();
}

hipError_t launch_win_compact(int prec, const MigSpecies &m, const int *stay, const int *pos,
                              const MigBuffers &sb, hipStream_t st) {
    if (m.np == 0) return hipSuccess;
    if (prec == 0)
        hipLaunchKernelGGL(k_win_compact<double>, dim3(nblocks(m.np, 256)), dim3(256), 0, st, m,
                           stay, pos, sb);
    else
        hipLaunchKernelGGL(k_win_compact<int>, dim3(nblocks(m.np, 256)), dim3(256), 0, st, m, stay,
                           pos, sb);
    return hipGetLastError();
}

hipError_t launch_win_fill(int prec, const MigSpecies &m, long long nstay, const MigBuffers &sb,
                           const MigSpecies &in, int zoff, int nz, int nxy, hipStream_t st) {
    const long long n = nstay + in.np;
    if (n == 0) return hipSuccess;
    if (prec == 0)
        hipLaunchKernelGGL((k_win_fill<double, 0>), dim3(nblocks(n, 256)), dim3(256), 0, st, m, nstay,
                           sb, in, zoff, nz, nxy);
    else
        hipLaunchKernelGGL((k_win_fill<int, 1>), dim3(nblocks(n, 256)), dim3(256), 0, st, m, nstay, sb,
                           in, zoff, nz, nxy);
    return hipGetLastError();
}

}  // namespace pic
