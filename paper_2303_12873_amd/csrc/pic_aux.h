// Host-side launchers of the libpic kernels (internal).
#pragma once

#include "pic_dev.h"

namespace pic {

hipError_t launch_tile_keys(int prec, const DevSpecies *spt, int s, long long np,
                            const DevBox *boxes, int *key, int *val, int *err, hipStream_t st);
size_t scan_scratch_ints(long long n);
hipError_t scan_exclusive(const int *in, int *out, long long n, int *total, int *scratch,
                          hipStream_t st);
int radix_blocks(long long n);
hipError_t radix_pass(const int *kin, const int *vin, int *kout, int *vout, long long n,
                      int shift, int *counts, int *scan_scratch, hipStream_t st);
hipError_t launch_tile_offsets(const int *key, long long n, int nkeys, int *off, hipStream_t st);
hipError_t launch_gather4(const void *src, const int *perm, void *dst, long long n, hipStream_t st);
hipError_t launch_gather8(const void *src, const int *perm, void *dst, long long n, hipStream_t st);
hipError_t launch_copy4(const void *src, void *dst, long long n, hipStream_t st);
hipError_t launch_copy8(const void *src, void *dst, long long n, hipStream_t st);
hipError_t launch_items(const DevSpecies *spt, const int *prefix, int nsp, int nslots, int chunk,
                        int *counts, int *starts, int *scan_scratch, Item *items, int *nitems,
                        int *queue, hipStream_t st);
hipError_t launch_set_int(int *p, int v, hipStream_t st);
hipError_t launch_zero_ints(int *p, int n, hipStream_t st);
hipError_t launch_zero_j(const DevFields &f, const DevBox *boxes, const long long *fp, int nb,
                         long long total, hipStream_t st);
hipError_t launch_fdtd(int prec, const DevFields &f, const DevBox *boxes, const long long *fp,
                       int nb, long long total, hipStream_t st);
hipError_t launch_div_edge(const DevBox *boxes, int bi, long long ncells, double *const v[3],
                           double *out, hipStream_t st);

// per-order particle kernels (pic_particles.hip built with PIC_ORDER = 1, 2, 3)
#define PIC_DECL_ORDER(N)                                                                        \
    hipError_t launch_particles_o##N(const KParams &prm, int prec, int form, int mode, int dims, \
                                     int grid, int block, size_t lds, int species,               \
                                     hipStream_t st);                                            \
    hipError_t particles_lds_limit_o##N(int prec, int bytes);                                    \
    hipError_t launch_rho_o##N(const KParams &prm, int prec, int species, long long np,          \
                               double *rho, hipStream_t st);
PIC_DECL_ORDER(1)
PIC_DECL_ORDER(2)
PIC_DECL_ORDER(3)
#undef PIC_DECL_ORDER

}  // namespace pic
