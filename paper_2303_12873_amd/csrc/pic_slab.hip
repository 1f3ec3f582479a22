// Decomposition of one periodic box into slabs along z, held as the boxes of
// one context: the data layout of the paper's multi-GPU runs (Sec. III.B:
// each GPU owns a part of the domain and exchanges guard regions and
// particles with its neighbours), exercised on one GPU.
//
// Slab s (box s of the context, s = 0 .. nslab-1 in z order) owns the global
// layers [z0_s, z0_s + nz_s) and stores them at local z in [g, g + nz_s),
// with g guard layers below ([0, g)) and above ([g + nz_s, 2 g + nz_s));
// every slab has the global box's nx, ny.  Neighbours are periodic: slab
// s - 1 of slab 0 is the last one.  Requirements (checked on the host):
// nz_s >= 2 g, so that the guard layers of one side come from one
// neighbour and the two boundary bands of an interior do not overlap.
//
// Per step (what a caller does, see libpic.h):
//   1. fill the E/B guards from the neighbours' interiors;
//   2. particle update on all slabs (the batched kernel covers every box in
//      one launch); J lands in interiors and guards;
//   3. add every guard's J into the owning neighbour's interior, then copy
//      the complete interior J back into the guards;
//   4. Yee update of every slab (the periodic wrap inside a slab box only
//      corrupts guard layers farther than 3 from the interior, and g >= 3);
//   5. move the particles that left a slab's interior to the neighbour.
#include <algorithm>

#include "pic_dev.h"
#include "pic_aux.h"

namespace pic {
namespace {

inline unsigned nblocks(long long n, int bs) { return (unsigned)((n + bs - 1) / bs); }

__device__ inline long long slab_index(const DevBox &b, int i, int j, int z) {
    return b.cell_base + i + (long long)b.n[0] * (j + (long long)b.n[1] * z);
}

// Guard fill: thread -> (slab, side band of g layers, layer, cell of the
// layer).  Low guard layer l of slab s <- layer nz_p + l of slab p = s - 1;
// high guard layer l <- layer g + l of slab q = s + 1.
template <typename T>
__global__ void k_slab_fill(SlabComps<T> f, int ncomp, const DevBox *boxes, int nslab, int g) {
    const DevBox &b0 = boxes[0];
    const long long nxy = (long long)b0.n[0] * b0.n[1];
    const long long per_slab = 2LL * g * nxy;
    long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= per_slab * nslab) return;
    const int s = (int)(t / per_slab);
    long long r = t - s * per_slab;
    const int band = (int)(r / (g * nxy));          // 0 low, 1 high
    r -= band * g * nxy;
    const int l = (int)(r / nxy);
    const long long c = r - l * nxy;
    const int i = (int)(c % b0.n[0]), j = (int)(c / b0.n[0]);
    const DevBox &bs = boxes[s];
    const int nz_s = bs.n[2] - 2 * g;
    long long dst, src;
    if (band == 0) {
        const int p = s == 0 ? nslab - 1 : s - 1;
        const DevBox &bp = boxes[p];
        dst = slab_index(bs, i, j, l);
        src = slab_index(bp, i, j, (bp.n[2] - 2 * g) + l);
    } else {
        const int q = s == nslab - 1 ? 0 : s + 1;
        dst = slab_index(bs, i, j, g + nz_s + l);
        src = slab_index(boxes[q], i, j, g + l);
    }
    for (int k = 0; k < ncomp; ++k) f.c[k][dst] = f.c[k][src];
}

// J guard reduction (pull, deterministic): interior layer g + l of slab s
// (bottom band) adds the high guard layer g + nz_p + l of slab p = s - 1;
// interior layer nz_s + l (top band) adds the low guard layer l of slab
// q = s + 1.
__global__ void k_slab_sum_j(SlabComps<double> f, const DevBox *boxes, int nslab, int g) {
    const DevBox &b0 = boxes[0];
    const long long nxy = (long long)b0.n[0] * b0.n[1];
    const long long per_slab = 2LL * g * nxy;
    long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= per_slab * nslab) return;
    const int s = (int)(t / per_slab);
    long long r = t - s * per_slab;
    const int band = (int)(r / (g * nxy));
    r -= band * g * nxy;
    const int l = (int)(r / nxy);
    const long long c = r - l * nxy;
    const int i = (int)(c % b0.n[0]), j = (int)(c / b0.n[0]);
    const DevBox &bs = boxes[s];
    const int nz_s = bs.n[2] - 2 * g;
    long long dst, src;
    if (band == 0) {
        const int p = s == 0 ? nslab - 1 : s - 1;
        const DevBox &bp = boxes[p];
        dst = slab_index(bs, i, j, g + l);
        src = slab_index(bp, i, j, g + (bp.n[2] - 2 * g) + l);
    } else {
        const int q = s == nslab - 1 ? 0 : s + 1;
        dst = slab_index(bs, i, j, nz_s + l);
        src = slab_index(boxes[q], i, j, l);
    }
    for (int k = 0; k < 3; ++k) f.c[k][dst] += f.c[k][src];
}

// ---------------------------------------------------------------- migration

// Direction of every particle: 0 stays, 1 left through the low face, 2
// through the high face (local z below g, or at or above g + nz).
template <int PREC>
__global__ void k_mig_flags(MigSpecies m, int g, int nzs, int nxy, int *stay, int *down,
                            int *up) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m.np) return;
    int z;
    if (PREC == 0) z = (int)floor(((const double *)m.a[m.zi])[i]);
    else z = ((const int *)m.a[0])[i] / nxy;
    const int d = z < g ? 1 : (z >= g + nzs ? 2 : 0);
    stay[i] = d == 0;
    down[i] = d == 1;
    up[i] = d == 2;
}

// Stayers to the staging arrays (compacted, in order); leavers to the send
// arrays of their direction, with z moved into the destination's frame
// (down: + nz of the lower slab; up: - nz of this slab).
template <typename E, int PREC>
__global__ void k_mig_scatter(MigSpecies m, const int *stay, const int *down, const int *up,
                              const int *pst, const int *pdn, const int *pup, MigBuffers sb,
                              int shift_down, int shift_up, int nxy) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m.np) return;
    E *dst[MIG_ARRAYS];
    long long k;
    int shift = 0;
    if (stay[i]) {
        k = pst[i];
        for (int a = 0; a < m.na; ++a) dst[a] = (E *)sb.stay[a];
    } else if (down[i]) {
        k = pdn[i];
        shift = shift_down;
        for (int a = 0; a < m.na; ++a) dst[a] = (E *)sb.down[a];
    } else {
        k = pup[i];
        shift = -shift_up;
        for (int a = 0; a < m.na; ++a) dst[a] = (E *)sb.up[a];
        (void)up;
    }
    for (int a = 0; a < m.na; ++a) {
        E v = ((const E *)m.a[a])[i];
        if (shift != 0) {
            if (PREC == 0 && a == m.zi) v = (E)((double)v + (double)shift);
            if (PREC == 1 && a == 0) v = (E)((int)v + shift * nxy);
        }
        dst[a][k] = v;
    }
}

// Species arrays <- stayers, then the arrivals from below (the lower slab's
// up-send), then from above (the upper slab's down-send).
template <typename E>
__global__ void k_mig_gather(MigSpecies m, long long nstay, MigBuffers own, long long nlow,
                             MigBuffers low, long long nhigh, MigBuffers high) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long n = nstay + nlow + nhigh;
    if (i >= n) return;
    for (int a = 0; a < m.na; ++a) {
        E v;
        if (i < nstay) v = ((const E *)own.stay[a])[i];
        else if (i < nstay + nlow) v = ((const E *)low.up[a])[i - nstay];
        else v = ((const E *)high.down[a])[i - nstay - nlow];
        ((E *)m.a[a])[i] = v;
    }
}

}  // namespace

hipError_t launch_slab_fill(int prec, void *const *comps, int ncomp, const DevBox *boxes,
                            int nslab, int g, long long nxy, hipStream_t st) {
    const long long n = 2LL * g * nxy * nslab;
    if (n == 0) return hipSuccess;
    if (prec == 0) {
        SlabComps<double> f;
        for (int k = 0; k < ncomp; ++k) f.c[k] = (double *)comps[k];
        hipLaunchKernelGGL(k_slab_fill<double>, dim3(nblocks(n, 256)), dim3(256), 0, st, f, ncomp,
                           boxes, nslab, g);
    } else {
        SlabComps<float> f;
        for (int k = 0; k < ncomp; ++k) f.c[k] = (float *)comps[k];
        hipLaunchKernelGGL(k_slab_fill<float>, dim3(nblocks(n, 256)), dim3(256), 0, st, f, ncomp,
                           boxes, nslab, g);
    }
    return hipGetLastError();
}

hipError_t launch_slab_sum_j(double *const J[3], const DevBox *boxes, int nslab, int g,
                             long long nxy, hipStream_t st) {
    const long long n = 2LL * g * nxy * nslab;
    if (n == 0) return hipSuccess;
    SlabComps<double> f;
    for (int k = 0; k < 3; ++k) f.c[k] = J[k];
    hipLaunchKernelGGL(k_slab_sum_j, dim3(nblocks(n, 256)), dim3(256), 0, st, f, boxes, nslab, g);
    return hipGetLastError();
}

hipError_t launch_mig_flags(int prec, const MigSpecies &m, int g, int nzs, int nxy, int *stay,
                            int *down, int *up, hipStream_t st) {
    if (m.np == 0) return hipSuccess;
    if (prec == 0)
        hipLaunchKernelGGL(k_mig_flags<0>, dim3(nblocks(m.np, 256)), dim3(256), 0, st, m, g, nzs,
                           nxy, stay, down, up);
    else
        hipLaunchKernelGGL(k_mig_flags<1>, dim3(nblocks(m.np, 256)), dim3(256), 0, st, m, g, nzs,
                           nxy, stay, down, up);
    return hipGetLastError();
}

hipError_t launch_mig_scatter(int prec, const MigSpecies &m, const int *stay, const int *down,
                              const int *up, const int *pst, const int *pdn, const int *pup,
                              const MigBuffers &sb, int shift_down, int shift_up, int nxy,
                              hipStream_t st) {
    if (m.np == 0) return hipSuccess;
    if (prec == 0)
        hipLaunchKernelGGL((k_mig_scatter<double, 0>), dim3(nblocks(m.np, 256)), dim3(256), 0, st,
                           m, stay, down, up, pst, pdn, pup, sb, shift_down, shift_up, nxy);
    else
        hipLaunchKernelGGL((k_mig_scatter<int, 1>), dim3(nblocks(m.np, 256)), dim3(256), 0, st, m,
                           stay, down, up, pst, pdn, pup, sb, shift_down, shift_up, nxy);
    return hipGetLastError();
}

hipError_t launch_mig_gather(int prec, const MigSpecies &m, long long nstay, const MigBuffers &own,
                             long long nlow, const MigBuffers &low, long long nhigh,
                             const MigBuffers &high, hipStream_t st) {
    const long long n = nstay + nlow + nhigh;
    if (n == 0) return hipSuccess;
    if (prec == 0)
        hipLaunchKernelGGL(k_mig_gather<double>, dim3(nblocks(n, 256)), dim3(256), 0, st, m, nstay,
                           own, nlow, low, nhigh, high);
    else
        hipLaunchKernelGGL(k_mig_gather<int>, dim3(nblocks(n, 256)), dim3(256), 0, st, m, nstay,
                           own, nlow, low, nhigh, high);
    return hipGetLastError();
}

}  // namespace pic
