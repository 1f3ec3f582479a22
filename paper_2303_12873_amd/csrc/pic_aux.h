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
// Rank-major keys: from sorted (tile << cbits | cell) keys, key2 = tile <<
// rbits | min(rank within the cell's run, 2^rbits - 1).  Scratch: heads,
// starts (n ints each), total (1 int).
// Rank-major order inside every tile from keys sorted by tile (stable) whose
// low cbits hold the cell within the tile (V cells, at most RM_MAXV): ranks
// 0 .. RM_RMAX - 1 one per occupied cell, the rest last, by cell; perm_out
// = perm_in reordered; rank_tmp: n ints of scratch.
constexpr int RM_RMAX = 15;
constexpr int RM_MAXV = 1024;
hipError_t rank_major_tiles(const int *key, const int *perm_in, const int *off, int nkeys,
                            int cbits, int V, int *rank_tmp, int *perm_out, hipStream_t st);
hipError_t rank_keys(const int *key, long long n, int cbits, int rbits, int *heads, int *starts,
                     int *key2, int *total, int *scan_scratch, hipStream_t st);
hipError_t launch_copy4(const void *src, void *dst, long long n, hipStream_t st);
// Permute narr particle arrays of elem_bytes (4 or 8) each through perm
// (dst[i] = src[perm[i]], in place) in groups that share one read of perm:
// stage holds PERM_GROUP_BYTES per element.
constexpr int PERM_GROUP_BYTES = 32;
hipError_t launch_permute(int elem_bytes, void *const *arrays, int narr, const int *perm,
                          void *stage, long long n, hipStream_t st);
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
// Energies (FP64, a check).  EnergySp: one species' momenta and weights
// (device pointers, the context's precision), count and mass.  Deterministic
// two-pass reduction: per-block partials in `part` (energy_scratch_doubles
// (nsp) doubles, fully overwritten where read), then out[0] = 1/2 sum E.E dV,
// out[1] = 1/2 sum B.B dV over box bi, out[2 + s] = sum w m (gamma - 1) of
// sps[s] (0 when np == 0).  nsp <= ENERGY_MAX_SPECIES.
constexpr int ENERGY_MAX_SPECIES = 16;
constexpr int ENERGY_MAX_GRID = 1024;
struct EnergySp {
    const void *u[3];
    const void *w;
    long long np;
    double m;
};
struct EnergyPlan {
    int nout;
    int off[2 + ENERGY_MAX_SPECIES], cnt[2 + ENERGY_MAX_SPECIES], str[2 + ENERGY_MAX_SPECIES];
};
size_t energy_scratch_doubles(int nsp);
hipError_t launch_energy(int prec, const DevFields &f, const DevBox *boxes, int bi,
                         long long ncells, const EnergySp *sps, int nsp, double *part,
                         double *out, hipStream_t st);
// Per-layer moments along z of species s into out (5 doubles per layer,
// added; see k_slice_moments).
hipError_t launch_slice_moments(int prec, const DevSpecies *spt, int s, long long np,
                                const DevBox *boxes, double *out, hipStream_t st);
hipError_t launch_zero_doubles(double *p, long long n, hipStream_t st);
hipError_t launch_div_edge(const DevBox *boxes, int bi, long long ncells, double *const v[3],
                           double *out, hipStream_t st);

// z-slab decomposition (pic_slab.hip).  SlabComps: field component
// pointers (E/B: 6 or 3, J: 3).  MigSpecies: the particle arrays of one
// species of one slab (FP64: x, u, w with zi the index of x[2]; split: cell
// first, then offsets, u, w; NULL arrays left out), all 8 or 4 bytes per
// particle.  MigBuffers: staging (stay) and send (down / up) arrays of the
// same layout.
constexpr int MIG_ARRAYS = 8;
template <typename T> struct SlabComps {
    T *c[6];
};
struct MigSpecies {
    void *a[MIG_ARRAYS];
    int na;
    int zi;
    long long np;
};
struct MigBuffers {
    void *stay[MIG_ARRAYS];
    void *down[MIG_ARRAYS];
    void *up[MIG_ARRAYS];
};
hipError_t launch_slab_fill(int prec, void *const *comps, int ncomp, const DevBox *boxes,
                            int nslab, int g, long long nxy, hipStream_t st);
hipError_t launch_slab_sum_j(double *const J[3], const DevBox *boxes, int nslab, int g,
                             long long nxy, hipStream_t st);
hipError_t launch_mig_flags(int prec, const MigSpecies &m, int g, int nzs, int nxy, int *stay,
                            int *down, int *up, hipStream_t st);
hipError_t launch_mig_scatter(int prec, const MigSpecies &m, const int *stay, const int *down,
                              const int *up, const int *pst, const int *pdn, const int *pup,
                              const MigBuffers &sb, int shift_down, int shift_up, int nxy,
                              hipStream_t st);
hipError_t launch_mig_gather(int prec, const MigSpecies &m, long long nstay, const MigBuffers &own,
                             long long nlow, const MigBuffers &low, long long nhigh,
                             const MigBuffers &high, hipStream_t st);

// Boundaries (pic_bound.hip): laser antenna, moving window.
struct AntennaArgs {
    int k;                 // window-frame cell layer of the sheet
    double E0, omega, waist, x0, y0, t0, tau;
};
hipError_t launch_antenna(double *Jx, const DevBox *boxes, int bi, long long nxy,
                          const AntennaArgs &an, double t, hipStream_t st);
hipError_t launch_zero_layer(int prec, void *const *comps, const DevBox *boxes, int bi, long long nxy,
                             int k, hipStream_t st);
hipError_t launch_box_zoff(DevBox *boxes, int bi, int zoff, hipStream_t st);
hipError_t launch_win_flags(int prec, const MigSpecies &m, int k, int nxy, int *stay,
                            hipStream_t st);
hipError_t launch_win_compact(int prec, const MigSpecies &m, const int *stay, const int *pos,
                              const MigBuffers &sb, hipStream_t st);
hipError_t launch_win_fill(int prec, const MigSpecies &m, long long nstay, const MigBuffers &sb,
                           const MigSpecies &in, int zoff, int nz, int nxy, hipStream_t st);

// Electrostatic variant (pic_es.hip): Poisson by conjugate gradients, E =
// -grad phi, particle update in E alone.
constexpr int ES_DOT_GRID = 1024;
hipError_t launch_neg_lap(const DevBox *boxes, int bi, long long n, const double *x, double *y,
                          hipStream_t st);
hipError_t launch_dot(const double *a, const double *b, long long n, double *part, double *out,
                      hipStream_t st);
hipError_t launch_remove_mean(double *x, long long n, double *part, double *sc, const double *ones,
                              hipStream_t st);
hipError_t launch_cg_xr(double *x, double *r, const double *p, const double *ap, long long n,
                        const double *sc, hipStream_t st);
hipError_t launch_cg_p(double *p, const double *r, long long n, const double *sc, hipStream_t st);
hipError_t launch_copy_scalar(double *sc, int to, int from, hipStream_t st);
hipError_t launch_copy_d(const double *a, double *b, long long n, hipStream_t st);
hipError_t launch_zero_d(double *a, long long n, hipStream_t st);
hipError_t launch_es_field(int prec, const DevBox *boxes, int bi, long long n, const double *phi,
                           const DevFields &f, hipStream_t st);
hipError_t launch_es_push(int order, int prec, const DevSpecies *spt, int s, long long np,
                          const DevBox *boxes, const DevFields &f, int *err, hipStream_t st);

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
