// Host-side launchers of the libpic kernels (internal).
#pragma once

#include "pic_dev.h"

namespace pic {

// Sort keys: the tile id, or with cbits > 0 (tile id, cell class, cell in
// tile) packed as tile << (cbits + 2) | class << cbits | cell (classes != 0)
// or tile << cbits | cell (classes == 0).
hipError_t launch_tile_keys(int prec, const DevSpecies *spt, int s, long long np,
                            const DevBox *boxes, int cbits, int classes, int *key, int *val,
                            int *err, hipStream_t st);
size_t scan_scratch_ints(long long n);
hipError_t scan_exclusive(const int *in, int *out, long long n, int *total, int *scratch,
                          hipStream_t st);
int radix_blocks(long long n);
hipError_t radix_pass(const int *kin, const int *vin, int *kout, int *vout, long long n,
                      int shift, int *counts, int *scan_scratch, hipStream_t st);
hipError_t launch_tile_offsets(const int *key, long long n, int nkeys, int shift, int *off,
                              hipStream_t st);
hipError_t launch_shift_copy(const int *src, int *dst, long long n, int shift, hipStream_t st);
// Stable reorder of each tile's cell-ordered particles: whole groups of four
// of a cell first, each cell's last (count mod 4) after them.  key: sorted
// keys (tile = key >> shift), perm_in: their source indices; perm_out gets
// the reordered source indices.  Scratch: work (n ints), work2 (2n ints),
// totals (2 ints); perm_out must not alias the inputs.
hipError_t quads_first(const int *key, const int *perm_in, long long n, int shift,
                       const int *tile_off, int *work, int *work2, int *perm_out, int *totals,
                       int *scan_scratch, hipStream_t st);
hipError_t launch_gather4(const void *src, const int *perm, void *dst, long long n, hipStream_t st);
hipError_t launch_gather8(const void *src, const int *perm, void *dst, long long n, hipStream_t st);
hipError_t launch_copy4(const void *src, void *dst, long long n, hipStream_t st);
hipError_t launch_copy8(const void *src, void *dst, long long n, hipStream_t st);
// Work items of the batched kernel over the box-tile slots (bprefix: nb + 1
// tile-count prefix over the boxes; box_sp_off / box_sp: species per box).
hipError_t launch_items(const DevSpecies *spt, const int *bprefix, int nb, const int *box_sp_off,
                        const int *box_sp, int nslots, int chunk, int *counts, int *starts,
                        int *scan_scratch, Item *items, int *nitems, int *queue, hipStream_t st);
hipError_t launch_set_int(int *p, int v, hipStream_t st);
hipError_t launch_stamp(long long *out, hipStream_t st);
hipError_t launch_zero_ints(int *p, int n, hipStream_t st);
hipError_t launch_zero_j(const DevFields &f, const DevBox *boxes, const long long *fp, int nb,
                         long long total, hipStream_t st);
hipError_t launch_fdtd(int prec, const DevFields &f, const DevBox *boxes, const long long *fp,
                       int nb, long long total, hipStream_t st);
// Energies (FP64, a check): out[0] = 1/2 sum E.E dV, out[1] = 1/2 sum B.B dV
// over the cells of box bi, out[2 + s] = sum w m (gamma - 1) of species s
// with np[s] > 0 (np: host array), else 0.  out is zeroed first.
hipError_t launch_energy(int prec, const DevFields &f, const DevBox *boxes, int bi,
                         long long ncells, const DevSpecies *spt, const long long *np, int nsp,
                         double *out, int cus, hipStream_t st);
hipError_t launch_div_edge(const DevBox *boxes, int bi, long long ncells, double *const v[3],
                           double *out, hipStream_t st);

// Particle kernels: pic_particles.hip is compiled once per (shape order N,
// precision P: 0 FP64, 1 split, part T): T = 0 holds the direct and
// straggler kernels, the push-only / deposit-only tiled kernels and the
// charge-density check; T = 1 the fused tiled kernels (one workgroup per
// tile); T = 2 the fused persistent (batched) kernels.
#define PIC_DECL_UNIT(N, P, T)                                                                   \
    hipError_t launch_particles_o##N##_p##P##_t##T(const KParams &prm, int form, int mode,       \
                                                   int dims, int grid, int block, size_t lds,    \
                                                   int species, hipStream_t st);                 \
    hipError_t particles_lds_limit_o##N##_p##P##_t##T(int bytes);
#define PIC_DECL_RHO(N, P)                                                                       \
    hipError_t launch_rho_o##N##_p##P##_t0(const KParams &prm, int species, long long np,       \
                                           double *rho, hipStream_t st);
#define PIC_DECL_ORDER(N)                                                                        \
    PIC_DECL_UNIT(N, 0, 0) PIC_DECL_UNIT(N, 0, 1) PIC_DECL_UNIT(N, 0, 2)                         \
    PIC_DECL_UNIT(N, 1, 0) PIC_DECL_UNIT(N, 1, 1) PIC_DECL_UNIT(N, 1, 2)                         \
    PIC_DECL_RHO(N, 0) PIC_DECL_RHO(N, 1)
PIC_DECL_ORDER(1)
PIC_DECL_ORDER(2)
PIC_DECL_ORDER(3)
#undef PIC_DECL_ORDER
#undef PIC_DECL_RHO
#undef PIC_DECL_UNIT

using ParticleLauncher = hipError_t (*)(const KParams &, int, int, int, int, int, size_t, int,
                                        hipStream_t);
using LdsLimiter = hipError_t (*)(int);
using RhoLauncher = hipError_t (*)(const KParams &, int, long long, double *, hipStream_t);

}  // namespace pic
