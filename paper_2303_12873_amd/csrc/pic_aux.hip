// Non-particle kernels of libpic: the per-tile stable counting sort (LSD
// radix passes of 8 bits over the tile id, each pass a stable counting sort),
// device-wide exclusive scan, per-tile offsets, permutation of the particle
// arrays, work-item list of the batched kernel, J zeroing, the Yee FDTD
// update over all boxes, and the node divergence used by the continuity
// check.
#include <algorithm>

#include "pic_dev.h"
#include "pic_math.h"
#include "pic_aux.h"

namespace pic {
namespace {

constexpr int SBS = 256;           // sort/scan block size (4 waves)
constexpr int SIPT = 16;           // sort items per thread
constexpr int SITEMS = SBS * SIPT; // elements per sort block
constexpr int SCAN_IPT = 4;
constexpr int SCAN_ITEMS = SBS * SCAN_IPT;

__device__ inline int lane_id() { return threadIdx.x & 63; }
__device__ inline int wave_id() { return threadIdx.x >> 6; }

// ------------------------------------------------------------ keys

template <int PREC>
__global__ void k_tile_keys(const DevSpecies *spt, int s, const DevBox *boxes, int cbits,
                            int classes, int *key, int *val, int *err) {
    const DevSpecies &sp = spt[s];
    const DevBox &b = boxes[sp.box];
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= sp.np) return;
    int c[3] = {0, 0, 0};
    bool ok = true;
    if (PREC == 0) {
        #pragma unroll
        for (int d = 0; d < 3; ++d) {
            if (b.dim == 2 && d == 1) continue;
            double x = sp.x[d][i];
            if (!(x >= 0.0 && x < (double)b.n[d])) { ok = false; break; }
            c[d] = (int)floor(x);
        }
    } else {
        int cell = sp.cell[i];
        if (cell < 0 || (long long)cell >= b.ncells) ok = false;
        else {
            int nxy = b.n[0] * b.n[1];
            c[2] = cell / nxy;
            int r = cell - c[2] * nxy;
            c[1] = r / b.n[0];
            c[0] = r - c[1] * b.n[0];
        }
    }
    int k;
    if (ok) {
        const int tx = c[0] / b.tile[0], ty = c[1] / b.tile[1], tz = c[2] / b.tile[2];
        k = tx + b.nt[0] * (ty + b.nt[1] * tz);
        if (cbits > 0) {
            const int lx = c[0] - tx * b.tile[0], ly = c[1] - ty * b.tile[1],
                      lz = c[2] - tz * b.tile[2];
            const int within = lx + b.tile[0] * (ly + (b.dim == 3 ? b.tile[1] : 1) * lz);
            if (classes) k = (k << (cbits + 2)) | (((lx + ly + lz) & 3) << cbits) | within;
            else k = (k << cbits) | within;
        }
    } else {
        // bucket of invalid particles, after every tile
        k = cbits > 0 ? (b.ntiles << (cbits + (classes ? 2 : 0))) : b.ntiles;
        atomicOr(err, 1);
    }
    key[i] = k;
    val[i] = (int)i;
}

// ------------------------------------------------------------ radix passes

// Lanes of this wave whose 8-bit digit equals ours (among valid lanes).
// Fast path: every valid lane holds the first lane's digit (the common case
// in the passes after the first, the keys being nearly sorted by tile).
__device__ inline unsigned long long peers(int digit, bool valid) {
    unsigned long long m = __ballot(valid);
    const int d0 = __builtin_amdgcn_readfirstlane(digit);
    if (__ballot(valid && digit == d0) == m) return m;
#pragma unroll
    for (int b = 0; b < 8; ++b) {
        int bit = (digit >> b) & 1;
        unsigned long long bal = __ballot(bit);
        m &= bit ? bal : ~bal;
    }
    return m;
}

__global__ void __launch_bounds__(SBS) k_radix_up(const int *key, long long n, int shift,
                                                  int *counts, int nblocks) {
    __shared__ int hist[256];
    hist[threadIdx.x] = 0;
    __syncthreads();
    const long long base = (long long)blockIdx.x * SITEMS;
    const unsigned long long below = (1ull << lane_id()) - 1ull;
    for (int r = 0; r < SIPT; ++r) {
        long long e = base + (long long)r * SBS + threadIdx.x;
        bool valid = e < n;
        int d = valid ? ((key[e] >> shift) & 255) : 0;
        unsigned long long m = peers(d, valid);
        if (valid && (m & below) == 0ull) atomicAdd(&hist[d], __popcll(m));
    }
    __syncthreads();
    counts[(long long)threadIdx.x * nblocks + blockIdx.x] = hist[threadIdx.x];
}

__global__ void __launch_bounds__(SBS) k_radix_down(const int *key_in, const int *val_in,
                                                    int *key_out, int *val_out, long long n,
                                                    int shift, const int *offsets, int nblocks) {
    __shared__ int run[256];
    __shared__ int wcnt[SBS / 64][256];
    run[threadIdx.x] = offsets[(long long)threadIdx.x * nblocks + blockIdx.x];
    for (int w = 0; w < SBS / 64; ++w) wcnt[w][threadIdx.x] = 0;
    __syncthreads();
    const long long base = (long long)blockIdx.x * SITEMS;
    const int lane = lane_id(), wave = wave_id();
    const unsigned long long below = (1ull << lane) - 1ull;
    for (int r = 0; r < SIPT; ++r) {
        long long e = base + (long long)r * SBS + threadIdx.x;
        bool valid = e < n;
        int k = valid ? key_in[e] : 0;
        int v = valid ? val_in[e] : 0;
        int d = (k >> shift) & 255;
        unsigned long long m = peers(d, valid);
        int rank = __popcll(m & below);
        if (valid && rank == 0) wcnt[wave][d] = __popcll(m);
        __syncthreads();
        if (valid) {
            int pos = run[d] + rank;
            for (int w = 0; w < wave; ++w) pos += wcnt[w][d];
            key_out[pos] = k;
            val_out[pos] = v;
        }
        __syncthreads();
        int tot = 0;
        for (int w = 0; w < SBS / 64; ++w) { tot += wcnt[w][threadIdx.x]; wcnt[w][threadIdx.x] = 0; }
        run[threadIdx.x] += tot;
        __syncthreads();
    }
}

// offsets[t] = first sorted position whose tile (key >> shift) is >= t,
// t = 0 .. nkeys.
__global__ void k_tile_offsets(const int *key, long long n, int nkeys, int shift, int *off) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i > n) return;
    int prev = (i == 0) ? -1 : (key[i - 1] >> shift);
    int cur = (i == n) ? nkeys : (key[i] >> shift);
    for (int t = prev + 1; t <= cur; ++t) off[t] = (int)i;
}

__global__ void k_shift_copy(const int *src, int *dst, long long n, int shift) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = src[i] >> shift;
}

// ------------------------------------------------------------ quads first
//
// After the cell-ordered sort, the particles of one cell form a run of equal
// keys.  Each tile's particles are reordered (stably) so that the runs'
// whole groups of four come first and the last (count mod 4) particles of
// every run after them: every aligned group of four in the first part then
// shares one cell.

__device__ inline int run_head(const int *key, long long i) {
    return (i == 0 || key[i] != key[i - 1]) ? 1 : 0;
}

__global__ void k_run_heads(const int *key, long long n, int *h) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) h[i] = run_head(key, i);
}

// heads_excl: exclusive scan of the heads, i.e. the run index of a head.
__global__ void k_run_starts(const int *key, long long n, const int *heads_excl, int *starts) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && run_head(key, i)) starts[heads_excl[i]] = (int)i;
}

// Keys of the rank-major order: the tile of a sorted (tile, cell) key and
// the particle's rank within its run of equal keys (its cell), capped at
// 2^rbits - 1: key2 = tile << rbits | rank.
__global__ void k_rank_keys(const int *key, long long n, const int *heads_excl, const int *starts,
                            int cbits, int rbits, int *key2) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int r = heads_excl[i] + run_head(key, i) - 1;
    const int rmax = (1 << rbits) - 1;
    const int rank = (int)min(i - (long long)starts[r], (long long)rmax);
    key2[i] = ((key[i] >> cbits) << rbits) | rank;
}

// Rank-major order inside each tile, one workgroup of RM_WAVES waves per
// tile (grid-stride over tiles).  key: sorted by tile, ties in previous
// order, low cbits = the cell within the tile; perm_in: previous index of
// each sorted element; off: tile offsets (nkeys + 1).  An element that is
// the k-th of its cell c (k counted in sorted order, so in previous order)
// goes, for k < RMAX, to off[t] + base[k] + (number of cells c' < c holding
// more than k elements), base[k] = number of elements of ranks below k; the
// elements of rank >= RMAX follow, by cell and then rank.  This is the
// stable sort by (tile, min(rank, RMAX), cell) of the previous order.
// rank_tmp: n ints of scratch.  LDS: cnt[V], per-wave chunk counts
// [RM_WAVES][V], occupancy prefixes [RMAX][V] ushorts, the excess prefix
// [V], base[RMAX + 1] and the level totals [RMAX + 1].
constexpr int RM_WAVES = 4;
constexpr int RM_BATCH = 8;   // chunks of 64 RM_WAVES elements loaded at once
__global__ void __launch_bounds__(64 * RM_WAVES)
k_rank_major_tiles(const int *key, const int *perm_in, const int *off, int nkeys, int cbits,
                   int V, int *rank_tmp, int *perm_out) {
    extern __shared__ int rm_lds[];
    const int stride = (V + 1) & ~1;
    int *cnt = rm_lds;
    int *wcnt = cnt + V;
    unsigned short *occ = (unsigned short *)(wcnt + RM_WAVES * V);
    int *exc = (int *)(occ + RM_RMAX * stride);
    int *base = exc + V;
    int *ltot = base + RM_RMAX + 1;
    const int tid = threadIdx.x, bs = blockDim.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int mask = (1 << cbits) - 1;
    const unsigned long long below = (1ull << lane) - 1ull;
    const int cpt = (V + 63) / 64;                 // cells per lane in the scans
    for (int t = blockIdx.x; t < nkeys; t += gridDim.x) {
        const int o0 = off[t], o1 = off[t + 1];
        if (o1 <= o0) continue;
        for (int c = tid; c < V; c += bs) cnt[c] = 0;
        for (int c = tid; c < RM_WAVES * V; c += bs) wcnt[c] = 0;
        __syncthreads();
        // ranks in sorted order, in batches of RM_BATCH chunks whose keys are
        // loaded first; in chunk i0 wave w takes [i0 + 64 w, i0 + 64 w + 64)
        for (int b0 = o0; b0 < o1; b0 += RM_BATCH * bs) {
          int kk[RM_BATCH];
#pragma unroll
          for (int u = 0; u < RM_BATCH; ++u) {
              const int i = b0 + u * bs + tid;
              kk[u] = i < o1 ? key[i] : 0;
          }
#pragma unroll
          for (int u = 0; u < RM_BATCH; ++u) {
            const int i0 = b0 + u * bs;
            if (i0 >= o1) break;
            const int i = i0 + tid;
            const bool valid = i < o1;
            const int c = valid ? (kk[u] & mask) : 0;
            unsigned long long m = __ballot(valid);
            const int c0 = __builtin_amdgcn_readfirstlane(c);
            if (__ballot(valid && c == c0) != m) {
                for (int b = 0; b < cbits; ++b) {
                    const int bit = (c >> b) & 1;
                    const unsigned long long bal = __ballot(bit);
                    m &= bit ? bal : ~bal;
                }
            }
            const bool lead = valid && (m & below) == 0ull;
            if (lead) wcnt[wave * V + c] = __popcll(m);
            __syncthreads();
            int r = 0;
            if (valid) {
                r = cnt[c] + __popcll(m & below);
                for (int w = 0; w < wave; ++w) r += wcnt[w * V + c];
            }
            __syncthreads();
            if (lead) {
                atomicAdd(&cnt[c], __popcll(m));
                wcnt[wave * V + c] = 0;
            }
            if (valid) rank_tmp[i] = r;
            __syncthreads();
          }
        }
        // occupancy prefixes per rank level and the excess prefix: wave w
        // takes the levels k = w mod RM_WAVES, then thread 0 adds up the
        // level totals
        {
            for (int k = wave; k <= RM_RMAX; k += RM_WAVES) {
                int sum = 0;
                for (int q = 0; q < cpt; ++q) {
                    const int c = lane * cpt + q;
                    if (c < V) sum += k < RM_RMAX ? (cnt[c] > k ? 1 : 0) : max(cnt[c] - RM_RMAX, 0);
                }
                // exclusive prefix over the wave's lanes
                int incl = sum;
#pragma unroll
                for (int d = 1; d < 64; d <<= 1) {
                    const int y = __shfl_up(incl, d);
                    if (lane >= d) incl += y;
                }
                int run = incl - sum;
                for (int q = 0; q < cpt; ++q) {
                    const int c = lane * cpt + q;
                    if (c >= V) break;
                    if (k < RM_RMAX) {
                        occ[k * stride + c] = (unsigned short)run;
                        run += cnt[c] > k ? 1 : 0;
                    } else {
                        exc[c] = run;
                        run += max(cnt[c] - RM_RMAX, 0);
                    }
                }
                const int tot = __shfl(incl, 63);
                if (lane == 0) ltot[k] = tot;
            }
        }
        __syncthreads();
        if (tid == 0) {
            int run_tot = 0;
            for (int k = 0; k <= RM_RMAX; ++k) { base[k] = run_tot; run_tot += ltot[k]; }
        }
        __syncthreads();
        // positions (element i read back by the thread that wrote its rank)
        for (int b0 = o0; b0 < o1; b0 += RM_BATCH * bs) {
            int kk[RM_BATCH], rr[RM_BATCH], pp[RM_BATCH];
#pragma unroll
            for (int u = 0; u < RM_BATCH; ++u) {
                const int i = b0 + u * bs + tid;
                kk[u] = 0; rr[u] = 0; pp[u] = 0;
                if (i < o1) { kk[u] = key[i]; rr[u] = rank_tmp[i]; pp[u] = perm_in[i]; }
            }
#pragma unroll
            for (int u = 0; u < RM_BATCH; ++u) {
                const int i = b0 + u * bs + tid;
                if (i >= o1) continue;
                const int c = kk[u] & mask;
                const int r = rr[u];
                const int pos = r < RM_RMAX ? base[r] + occ[r * stride + c]
                                            : base[RM_RMAX] + exc[c] + (r - RM_RMAX);
                perm_out[o0 + pos] = pp[u];
            }
        }
        __syncthreads();
    }
}

__global__ void k_quad_flags(const int *key, long long n, const int *heads_excl, const int *starts,
                             const int *nruns, int *flag) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int r = heads_excl[i] + run_head(key, i) - 1;
    const long long start = starts[r];
    const long long end = r + 1 < *nruns ? starts[r + 1] : n;
    const long long cnt = end - start;
    flag[i] = (i - start) >= cnt - (cnt & 3) ? 1 : 0;
}

// Final position of sorted element i inside its tile [o0, o1): unflagged
// elements first, flagged after them, each in sorted order.
__global__ void k_quad_scatter(const int *key, long long n, int shift, const int *tile_off,
                               const int *flag, const int *fexcl, const int *ftotal,
                               const int *perm_in, int *perm_out) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int t = key[i] >> shift;
    const long long o0 = tile_off[t], o1 = tile_off[t + 1];
    const int g0 = fexcl[o0];
    const int g1 = o1 < n ? fexcl[o1] : *ftotal;
    const long long fb = fexcl[i] - g0;
    const long long unflagged = (o1 - o0) - (g1 - g0);
    const long long pos = flag[i] ? o0 + unflagged + fb : i - fb;
    perm_out[pos] = perm_in[i];
}

// ------------------------------------------------------------ scan

__device__ inline int wave_incl_scan(int v) {
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        int t = __shfl_up(v, o, 64);
        if (lane_id() >= o) v += t;
    }
    return v;
}

// Exclusive scan of SCAN_ITEMS consecutive elements per block; block total
// to sums[blockIdx].
__global__ void __launch_bounds__(SBS) k_scan_block(const int *in, int *out, long long n,
                                                    int *sums) {
    __shared__ int buf[SCAN_ITEMS];
    __shared__ int wtot[SBS / 64];
    const long long base = (long long)blockIdx.x * SCAN_ITEMS;
    for (int r = 0; r < SCAN_IPT; ++r) {
        long long e = base + r * SBS + threadIdx.x;
        buf[r * SBS + threadIdx.x] = e < n ? in[e] : 0;
    }
    __syncthreads();
    int loc[SCAN_IPT];
    int t = 0;
    for (int r = 0; r < SCAN_IPT; ++r) { loc[r] = t; t += buf[threadIdx.x * SCAN_IPT + r]; }
    int inc = wave_incl_scan(t);
    if (lane_id() == 63) wtot[wave_id()] = inc;
    __syncthreads();
    int wpre = 0;
    for (int w = 0; w < wave_id(); ++w) wpre += wtot[w];
    int excl = wpre + inc - t;
    for (int r = 0; r < SCAN_IPT; ++r) buf[threadIdx.x * SCAN_IPT + r] = excl + loc[r];
    if (threadIdx.x == SBS - 1) sums[blockIdx.x] = excl + t;
    __syncthreads();
    for (int r = 0; r < SCAN_IPT; ++r) {
        long long e = base + r * SBS + threadIdx.x;
        if (e < n) out[e] = buf[r * SBS + threadIdx.x];
    }
}

__global__ void k_scan_add(int *out, long long n, const int *sums_scanned) {
    long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n) out[e] += sums_scanned[e / SCAN_ITEMS];
}

// total = last exclusive value + last input (n >= 1), or 0.
__global__ void k_scan_total(const int *in, const int *out, long long n, int *total) {
    *total = n > 0 ? out[n - 1] + in[n - 1] : 0;
}

// ------------------------------------------------------------ permutation

template <typename T>
__global__ void k_copy(const T *src, T *dst, long long n) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = src[i];
}

// Up to PERM_GROUP_BYTES / sizeof(T) particle arrays permuted together: one
// kernel gathers them through perm (read once) into consecutive slices of a
// staging buffer, one kernel copies every slice back.
template <typename T> struct PermSet {
    T *a[PERM_GROUP_BYTES / 4];
    int n;
};

template <typename T>
__global__ void k_permute_set(PermSet<T> ps, const int *perm, T *stage, long long n) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const long long j = perm[i];
    // every load before any store: the compiler cannot tell that the stores
    // leave the sources alone, and would otherwise wait for each load in turn
    constexpr int G = PERM_GROUP_BYTES / (int)sizeof(T);
    T v[G];
#pragma unroll
    for (int k = 0; k < G; ++k)
        if (k < ps.n) v[k] = ps.a[k][j];
#pragma unroll
    for (int k = 0; k < G; ++k)
        if (k < ps.n) stage[k * n + i] = v[k];
}

template <typename T>
__global__ void k_unstage_set(PermSet<T> ps, const T *stage, long long n) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    constexpr int G = PERM_GROUP_BYTES / (int)sizeof(T);
    T v[G];     // every load before any store (see k_permute_set)
#pragma unroll
    for (int k = 0; k < G; ++k)
        if (k < ps.n) v[k] = stage[k * n + i];
#pragma unroll
    for (int k = 0; k < G; ++k)
        if (k < ps.n) ps.a[k][i] = v[k];
}


// ------------------------------------------------------------ work items

// Box-tile slots: slot g is tile g - prefix[b] of box b (prefix over the
// boxes' tile counts, nb + 1 entries).
__device__ inline int slot_box(const int *prefix, int nb, int g) {
    int lo = 0, hi = nb - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (prefix[mid] <= g) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Items of one box tile: none if it is empty, one item over all its species
// if they hold at most `chunk` particles together, else chunks of at most
// `chunk` particles of one species each.
struct TileItems {
    int total, chunks;
};

__device__ inline TileItems tile_items(const DevSpecies *spt, const int *box_sp_off,
                                       const int *box_sp, int b, int t, int chunk) {
    TileItems r{0, 0};
    for (int k = box_sp_off[b]; k < box_sp_off[b + 1]; ++k) {
        const int *off = spt[box_sp[k]].tile_off;
        const int n = off[t + 1] - off[t];
        r.total += n;
        r.chunks += (n + chunk - 1) / chunk;
    }
    return r;
}

__global__ void k_item_count(const DevSpecies *spt, const int *bprefix, int nb,
                             const int *box_sp_off, const int *box_sp, int nslots, int chunk,
                             int *counts) {
    int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= nslots) return;
    const int b = slot_box(bprefix, nb, g);
    const TileItems ti = tile_items(spt, box_sp_off, box_sp, b, g - bprefix[b], chunk);
    counts[g] = ti.total == 0 ? 0 : (ti.total <= chunk ? 1 : ti.chunks);
}

__global__ void k_item_fill(const DevSpecies *spt, const int *bprefix, int nb,
                            const int *box_sp_off, const int *box_sp, int nslots, int chunk,
                            const int *starts, Item *items) {
    int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= nslots) return;
    const int b = slot_box(bprefix, nb, g);
    const int t = g - bprefix[b];
    const TileItems ti = tile_items(spt, box_sp_off, box_sp, b, t, chunk);
    int st = starts[g];
    if (ti.total == 0) return;
    if (ti.total <= chunk) {
        items[st] = Item{-1 - b, t, 0, ti.total};
        return;
    }
    for (int k = box_sp_off[b]; k < box_sp_off[b + 1]; ++k) {
        const int s = box_sp[k];
        const int *off = spt[s].tile_off;
        const int p0 = off[t], p1 = off[t + 1];
        for (int a = p0; a < p1; a += chunk) items[st++] = Item{s, t, a, min(p1, a + chunk)};
    }
}

__global__ void k_set_int(int *p, int v) { *p = v; }

// The device's constant-rate wall clock, by one thread (a timing stamp).
__global__ void k_stamp(long long *out) { out[threadIdx.x] = wall_clock64(); }

__global__ void k_zero_ints(int *p, int n) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

// ------------------------------------------------------------ fields

__device__ inline int box_of(const long long *fp, int nb, long long g) {
    int lo = 0, hi = nb - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (fp[mid] <= g) lo = mid; else hi = mid - 1;
    }
    return lo;
}

__global__ void k_zero_j(DevFields f, const DevBox *boxes, const long long *fp, int nb,
                         long long total) {
    long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= total) return;
    int b = box_of(fp, nb, g);
    long long c = boxes[b].cell_base + (g - fp[b]);
    f.J[0][c] = 0.0;
    f.J[1][c] = 0.0;
    f.J[2][c] = 0.0;
}

struct CellNbr {
    long long c, xp, yp, zp, xm, ym, zm;
};

__device__ inline CellNbr neighbours(const DevBox &b, long long local) {
    const int n0 = b.n[0], n1 = b.n[1], n2 = b.n[2];
    int i = (int)(local % n0);
    long long r = local / n0;
    int j = (int)(r % n1);
    int k = (int)(r / n1);
    int ip = (i + 1 == n0) ? 0 : i + 1, im = (i == 0) ? n0 - 1 : i - 1;
    int jp = (j + 1 == n1) ? 0 : j + 1, jm = (j == 0) ? n1 - 1 : j - 1;
    int kp = (k + 1 == n2) ? 0 : k + 1, km = (k == 0) ? n2 - 1 : k - 1;
    auto id = [&](int a, int bb, int cc) {
        return b.cell_base + a + (long long)n0 * (bb + (long long)n1 * cc);
    };
    return CellNbr{id(i, j, k), id(ip, j, k), id(i, jp, k), id(i, j, kp),
                   id(im, j, k), id(i, jm, k), id(i, j, km)};
}

// Conductivity of the absorbing layers at array height za (cell units) of
// box b: frame height (za - zoff) mod n_z, depth d into a layer of L cells,
// sigma_max (d / L)^p.
__device__ inline double absorb_sigma(const DevBox &b, double za) {
    const double nz = (double)b.n[2], L = (double)b.abs_cells;
    double z = za - (double)b.zoff;
    z -= nz * floor(z / nz);
    double d = 0.0;
    if (z < L) d = L - z;
    else if (z > nz - L) d = z - (nz - L);
    if (d <= 0.0) return 0.0;
    double r = d / L, p = r;
    for (int k = 1; k < b.abs_power; ++k) p *= r;
    return b.abs_sigma * (b.abs_power == 0 ? 1.0 : p);
}

// Decay factor and source weight of a sub-step tau: exp(-sigma tau) and
// (1 - exp(-sigma tau)) / sigma (tau when sigma = 0).
__device__ inline void absorb_coef(double sigma, double tau, double &al, double &be) {
    if (sigma == 0.0) { al = 1.0; be = tau; return; }
    al = exp(-sigma * tau);
    be = (1.0 - al) / sigma;
}

__device__ inline int cell_k(const DevBox &b, long long local) {
    return (int)(local / ((long long)b.n[0] * b.n[1]));
}

// B -= h curl E, curl E at the B points (Yee).  2D: no d/dy terms.  In the
// absorbing layers B <- exp(-sigma h) B - (1 - exp(-sigma h)) / sigma curl E,
// sigma at each component's own z (B_x, B_y at k + 1/2, B_z at k).
template <typename T>
__global__ void k_faraday(DevFields f, const DevBox *boxes, const long long *fp, int nb,
                          long long total, double hfrac) {
    long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= total) return;
    int bi = box_of(fp, nb, g);
    const DevBox &b = boxes[bi];
    CellNbr q = neighbours(b, g - fp[bi]);
    const T *Ex = (const T *)f.E[0], *Ey = (const T *)f.E[1], *Ez = (const T *)f.E[2];
    T *Bx = (T *)f.B[0], *By = (T *)f.B[1], *Bz = (T *)f.B[2];
    const T h = (T)(hfrac * b.dt);
    const T ix = (T)(1.0 / b.dx[0]), iy = (T)(1.0 / b.dx[1]), iz = (T)(1.0 / b.dx[2]);
    T ez = Ez[q.c], ey = Ey[q.c], ex = Ex[q.c];
    // the cell's B read with E, before any store (which the compiler cannot
    // tell apart from the sources, and would wait for load by load)
    const T bx = Bx[q.c], by = By[q.c], bz = Bz[q.c];
    T dEz_dy = T(0), dEx_dy = T(0);
    if (b.dim == 3) { dEz_dy = (Ez[q.yp] - ez) * iy; dEx_dy = (Ex[q.yp] - ex) * iy; }
    T cx = dEz_dy - (Ey[q.zp] - ey) * iz;
    T cy = (Ex[q.zp] - ex) * iz - (Ez[q.xp] - ez) * ix;
    T cz = (Ey[q.xp] - ey) * ix - dEx_dy;
    if (b.abs_cells > 0) {
        const int k = cell_k(b, g - fp[bi]);
        const double hh = hfrac * b.dt;
        double a1, b1, a0, b0;
        absorb_coef(absorb_sigma(b, k + 0.5), hh, a1, b1);
        absorb_coef(absorb_sigma(b, (double)k), hh, a0, b0);
        Bx[q.c] = (T)a1 * bx - (T)b1 * cx;
        By[q.c] = (T)a1 * by - (T)b1 * cy;
        Bz[q.c] = (T)a0 * bz - (T)b0 * cz;
        return;
    }
    Bx[q.c] = bx - h * cx;
    By[q.c] = by - h * cy;
    Bz[q.c] = bz - h * cz;
}

// E += dt (curl B - J), curl B at the E points.
template <typename T>
__global__ void k_ampere(DevFields f, const DevBox *boxes, const long long *fp, int nb,
                         long long total) {
    long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= total) return;
    int bi = box_of(fp, nb, g);
    const DevBox &b = boxes[bi];
    CellNbr q = neighbours(b, g - fp[bi]);
    T *Ex = (T *)f.E[0], *Ey = (T *)f.E[1], *Ez = (T *)f.E[2];
    const T *Bx = (const T *)f.B[0], *By = (const T *)f.B[1], *Bz = (const T *)f.B[2];
    const T dt = (T)b.dt;
    const T ix = (T)(1.0 / b.dx[0]), iy = (T)(1.0 / b.dx[1]), iz = (T)(1.0 / b.dx[2]);
    T bx = Bx[q.c], by = By[q.c], bz = Bz[q.c];
    // the cell's E and J read before any store (see k_faraday)
    const T ex = Ex[q.c], ey = Ey[q.c], ez = Ez[q.c];
    const T jx = (T)f.J[0][q.c], jy = (T)f.J[1][q.c], jz = (T)f.J[2][q.c];
    T dBz_dy = T(0), dBx_dy = T(0);
    if (b.dim == 3) { dBz_dy = (bz - Bz[q.ym]) * iy; dBx_dy = (bx - Bx[q.ym]) * iy; }
    T cx = dBz_dy - (by - By[q.zm]) * iz;
    T cy = (bx - Bx[q.zm]) * iz - (bz - Bz[q.xm]) * ix;
    T cz = (by - By[q.xm]) * ix - dBx_dy;
    if (b.abs_cells > 0) {
        // E_x, E_y at k, E_z at k + 1/2
        const int k = cell_k(b, g - fp[bi]);
        double a0, b0, a1, b1;
        absorb_coef(absorb_sigma(b, (double)k), b.dt, a0, b0);
        absorb_coef(absorb_sigma(b, k + 0.5), b.dt, a1, b1);
        Ex[q.c] = (T)a0 * ex + (T)b0 * (cx - jx);
        Ey[q.c] = (T)a0 * ey + (T)b0 * (cy - jy);
        Ez[q.c] = (T)a1 * ez + (T)b1 * (cz - jz);
        return;
    }
    Ex[q.c] = ex + dt * (cx - jx);
    Ey[q.c] = ey + dt * (cy - jy);
    Ez[q.c] = ez + dt * (cz - jz);
}

// Node divergence of an E-staggered vector field (FP64).
__global__ void k_div_edge(const DevBox *boxes, int bi, const double *vx, const double *vy,
                           const double *vz, double *out) {
    const DevBox &b = boxes[bi];
    long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= b.ncells) return;
    CellNbr q = neighbours(b, g);
    long long base = b.cell_base;
    double d = (vx[q.c] - vx[q.xm]) / b.dx[0] + (vz[q.c] - vz[q.zm]) / b.dx[2];
    if (b.dim == 3) d += (vy[q.c] - vy[q.ym]) / b.dx[1];
    out[q.c - base] = d;
}

// ------------------------------------------------------------ energies
//
// Two passes, deterministic: every block of the field and kinetic passes
// writes its partial sums into its own slot of a scratch array (no atomics),
// then one block adds each output's partials in slot order.

// Sum of v over a 256-thread block (4 waves: shuffle reduction in each
// wave, then the four wave sums through LDS); the result is valid in
// thread 0.
__device__ inline double block_sum256(double v, double *lds4) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    if (lane_id() == 0) lds4[wave_id()] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0) t = (lds4[0] + lds4[1]) + (lds4[2] + lds4[3]);
    __syncthreads();
    return t;
}

// Field energy partials of box bi: part[2 b] = 1/2 sum E.E dV and
// part[2 b + 1] = 1/2 sum B.B dV over block b's cells (FP64 sums; E, B in
// the context's precision).
template <typename T>
__global__ void __launch_bounds__(256) k_field_energy(DevFields f, const DevBox *boxes, int bi,
                                                       double *part) {
    __shared__ double red[4];
    const DevBox &b = boxes[bi];
    double se = 0.0, sb = 0.0;
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x; c < b.ncells; c += stride) {
        const long long g = b.cell_base + c;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const double e = (double)((const T *)f.E[k])[g];
            const double bb = (double)((const T *)f.B[k])[g];
            se += e * e;
            sb += bb * bb;
        }
    }
    const double hdv = 0.5 * b.dx[0] * b.dx[1] * b.dx[2];
    se = block_sum256(se, red);
    sb = block_sum256(sb, red);
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = se * hdv;
        part[2 * blockIdx.x + 1] = sb * hdv;
    }
}

// Kinetic energy partials of one species: part[b] = sum over block b's
// particles of w m (gamma - 1), gamma - 1 = u.u / (1 + gamma) (no
// cancellation at small |u|).
template <typename T>
__global__ void __launch_bounds__(256) k_kinetic_energy(EnergySp sp, double *part) {
    __shared__ double red[4];
    const T *u0 = (const T *)sp.u[0], *u1 = (const T *)sp.u[1], *u2 = (const T *)sp.u[2];
    const T *w = (const T *)sp.w;
    double acc = 0.0;
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < sp.np; i += stride) {
        const double a = u0[i], bq = u1[i], c = u2[i];
        const double uu = a * a + bq * bq + c * c;
        acc += (double)w[i] * (uu / (1.0 + sqrt(1.0 + uu)));
    }
    acc = block_sum256(acc, red);
    if (threadIdx.x == 0) part[blockIdx.x] = acc * sp.m;
}

// out[k] = sum of partials [off[k], off[k] + cnt[k]) with stride str[k]
// (field parts interleave E and B), in slot order.  One block of 64 lanes.
__global__ void k_energy_final(const double *part, EnergyPlan plan, double *out) {
    const int k = blockIdx.x;
    if (k >= plan.nout) return;
    double acc = 0.0;
    if (threadIdx.x == 0) {
        for (int i = 0; i < plan.cnt[k]; ++i) acc += part[plan.off[k] + (long long)i * plan.str[k]];
        out[k] = acc;
    }
}

// Per-layer moments along z (window frame) of one species: out[5 k + q] +=
// w, w u_x, w u_y, w u_z, w m (gamma - 1) of every particle in frame layer
// k (FP64 atomics; summation order unspecified).
template <int PREC>
__global__ void k_slice_moments(const DevSpecies *spt, int s, const DevBox *boxes, double *out) {
    const DevSpecies &sp = spt[s];
    const DevBox &b = boxes[sp.box];
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= sp.np) return;
    int k;
    double u0, u1, u2, w;
    if (PREC == 0) {
        k = (int)floor(sp.x[2][i]);
        u0 = ((const double *)sp.u[0])[i]; u1 = ((const double *)sp.u[1])[i];
        u2 = ((const double *)sp.u[2])[i]; w = ((const double *)sp.w)[i];
    } else {
        k = sp.cell[i] / (b.n[0] * b.n[1]);
        u0 = ((const float *)sp.u[0])[i]; u1 = ((const float *)sp.u[1])[i];
        u2 = ((const float *)sp.u[2])[i]; w = ((const float *)sp.w)[i];
    }
    const int nz = b.n[2];
    k = ((k - b.zoff) % nz + nz) % nz;
    const double uu = u0 * u0 + u1 * u1 + u2 * u2;
    double *o = out + 5LL * k;
    atomicAdd(o + 0, w);
    atomicAdd(o + 1, w * u0);
    atomicAdd(o + 2, w * u1);
    atomicAdd(o + 3, w * u2);
    atomicAdd(o + 4, w * sp.m * (uu / (1.0 + sqrt(1.0 + uu))));
}

__global__ void k_zero_doubles(double *p, long long n) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.0;
}

inline unsigned blocks_for(long long n, int bs) { return (unsigned)((n + bs - 1) / bs); }

template <typename T>
hipError_t permute_arrays(void *const *arrays, int narr, const int *perm, void *stage, long long n,
                          hipStream_t st) {
    constexpr int G = PERM_GROUP_BYTES / (int)sizeof(T);
    for (int g0 = 0; g0 < narr; g0 += G) {
        PermSet<T> ps{};
        ps.n = std::min(G, narr - g0);
        for (int k = 0; k < ps.n; ++k) ps.a[k] = (T *)arrays[g0 + k];
        hipLaunchKernelGGL(k_permute_set<T>, dim3(blocks_for(n, 256)), dim3(256), 0, st, ps, perm,
                           (T *)stage, n);
        hipLaunchKernelGGL(k_unstage_set<T>, dim3(blocks_for(n, 256)), dim3(256), 0, st, ps,
                           (const T *)stage, n);
    }
    return hipGetLastError();
}

}  // namespace

// ============================================================ host launchers

hipError_t launch_tile_keys(int prec, const DevSpecies *spt, int s, long long np,
                            const DevBox *boxes, int cbits, int classes, int *key, int *val,
                            int *err, hipStream_t st) {
    if (np == 0) return hipSuccess;
    if (prec == 0)
        hipLaunchKernelGGL(k_tile_keys<0>, dim3(blocks_for(np, 256)), dim3(256), 0, st, spt, s,
                           boxes, cbits, classes, key, val, err);
    else
        hipLaunchKernelGGL(k_tile_keys<1>, dim3(blocks_for(np, 256)), dim3(256), 0, st, spt, s,
                           boxes, cbits, classes, key, val, err);
    return hipGetLastError();
}

size_t scan_scratch_ints(long long n) {
    size_t tot = 0;
    while (n > 1) {
        long long nb = (n + SCAN_ITEMS - 1) / SCAN_ITEMS;
        tot += (size_t)nb + 64;
        n = nb;
    }
    return tot + 64;
}

// Exclusive scan of in[0..n) into out (may alias in? no: distinct buffers
// not required, the block pass reads before it writes its own range).
hipError_t scan_exclusive(const int *in, int *out, long long n, int *total, int *scratch,
                          hipStream_t st) {
    if (n <= 0) {
        if (total) hipLaunchKernelGGL(k_set_int, dim3(1), dim3(1), 0, st, total, 0);
        return hipGetLastError();
    }
    long long nb = (n + SCAN_ITEMS - 1) / SCAN_ITEMS;
    int *sums = scratch;
    int *rest = scratch + nb + 64;
    if (total) {
        // the total needs the unscanned last input; read it before out may alias in
        hipLaunchKernelGGL(k_copy<int>, dim3(1), dim3(1), 0, st, in + (n - 1), total, 1ll);
    }
    hipLaunchKernelGGL(k_scan_block, dim3((unsigned)nb), dim3(SBS), 0, st, in, out, n, sums);
    if (nb > 1) {
        hipError_t e = scan_exclusive(sums, sums, nb, nullptr, rest, st);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_scan_add, dim3(blocks_for(n, 256)), dim3(256), 0, st, out, n,
                           (const int *)sums);
    }
    if (total) {
        // total = last input (already in *total) + last exclusive output
        hipLaunchKernelGGL(k_scan_total, dim3(1), dim3(1), 0, st, (const int *)total,
                           (const int *)(out + (n - 1)), 1ll, total);
    }
    return hipGetLastError();
}

int radix_blocks(long long n) { return (int)((n + SITEMS - 1) / SITEMS); }

hipError_t radix_pass(const int *kin, const int *vin, int *kout, int *vout, long long n,
                      int shift, int *counts, int *scan_scratch, hipStream_t st) {
    int nb = radix_blocks(n);
    if (nb == 0) return hipSuccess;
    hipLaunchKernelGGL(k_radix_up, dim3(nb), dim3(SBS), 0, st, kin, n, shift, counts, nb);
    hipError_t e = scan_exclusive(counts, counts, (long long)nb * 256, nullptr, scan_scratch, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_radix_down, dim3(nb), dim3(SBS), 0, st, kin, vin, kout, vout, n, shift,
                       (const int *)counts, nb);
    return hipGetLastError();
}

hipError_t launch_tile_offsets(const int *key, long long n, int nkeys, int shift, int *off,
                              hipStream_t st) {
    hipLaunchKernelGGL(k_tile_offsets, dim3(blocks_for(n + 1, 256)), dim3(256), 0, st, key, n,
                       nkeys, shift, off);
    return hipGetLastError();
}

hipError_t quads_first(const int *key, const int *perm_in, long long n, int shift,
                       const int *tile_off, int *work, int *work2, int *perm_out, int *totals,
                       int *scan_scratch, hipStream_t st) {
    if (n == 0) return hipSuccess;
    const unsigned nb = blocks_for(n, 256);
    int *heads = work;              // n: heads, then their exclusive scan
    int *starts = perm_out;         // n: run starts (perm_out is written last)
    int *flag = work2, *fexcl = work2 + n;
    hipLaunchKernelGGL(k_run_heads, dim3(nb), dim3(256), 0, st, key, n, heads);
    hipError_t e = scan_exclusive(heads, heads, n, totals, scan_scratch, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_run_starts, dim3(nb), dim3(256), 0, st, key, n, (const int *)heads, starts);
    hipLaunchKernelGGL(k_quad_flags, dim3(nb), dim3(256), 0, st, key, n, (const int *)heads,
                       (const int *)starts, (const int *)totals, flag);
    e = scan_exclusive(flag, fexcl, n, totals + 1, scan_scratch, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_quad_scatter, dim3(nb), dim3(256), 0, st, key, n, shift, tile_off,
                       (const int *)flag, (const int *)fexcl, (const int *)(totals + 1), perm_in,
                       perm_out);
    return hipGetLastError();
}

hipError_t rank_keys(const int *key, long long n, int cbits, int rbits, int *heads, int *starts,
                     int *key2, int *total, int *scan_scratch, hipStream_t st) {
    if (n == 0) return hipSuccess;
    const unsigned nb = blocks_for(n, 256);
    hipLaunchKernelGGL(k_run_heads, dim3(nb), dim3(256), 0, st, key, n, heads);
    hipError_t e = scan_exclusive(heads, heads, n, total, scan_scratch, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_run_starts, dim3(nb), dim3(256), 0, st, key, n, (const int *)heads, starts);
    hipLaunchKernelGGL(k_rank_keys, dim3(nb), dim3(256), 0, st, key, n, (const int *)heads,
                       (const int *)starts, cbits, rbits, key2);
    return hipGetLastError();
}

hipError_t rank_major_tiles(const int *key, const int *perm_in, const int *off, int nkeys,
                            int cbits, int V, int *rank_tmp, int *perm_out, hipStream_t st) {
    if (V > RM_MAXV || V <= 0) return hipErrorInvalidValue;
    const size_t lds = (size_t)V * 4 * (1 + RM_WAVES) + (size_t)RM_RMAX * ((V + 1) & ~1) * 2 +
                       (size_t)V * 4 + 2 * (RM_RMAX + 1) * 4;
    const int grid = std::min(nkeys, 65536);
    hipLaunchKernelGGL(k_rank_major_tiles, dim3(grid), dim3(64 * RM_WAVES), lds, st, key, perm_in,
                       off, nkeys, cbits, V, rank_tmp, perm_out);
    return hipGetLastError();
}

hipError_t launch_shift_copy(const int *src, int *dst, long long n, int shift, hipStream_t st) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_shift_copy, dim3(blocks_for(n, 256)), dim3(256), 0, st, src, dst, n, shift);
    return hipGetLastError();
}

hipError_t launch_permute(int elem_bytes, void *const *arrays, int narr, const int *perm,
                          void *stage, long long n, hipStream_t st) {
    if (n == 0 || narr == 0) return hipSuccess;
    if (elem_bytes == 4) return permute_arrays<int>(arrays, narr, perm, stage, n, st);
    return permute_arrays<long long>(arrays, narr, perm, stage, n, st);
}

hipError_t launch_copy4(const void *src, void *dst, long long n, hipStream_t st) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_copy<int>, dim3(blocks_for(n, 256)), dim3(256), 0, st, (const int *)src,
                       (int *)dst, n);
    return hipGetLastError();
}

hipError_t launch_items(const DevSpecies *spt, const int *bprefix, int nb, const int *box_sp_off,
                        const int *box_sp, int nslots, int chunk, int *counts, int *starts,
                        int *scan_scratch, Item *items, int *nitems, int *queue, hipStream_t st) {
    hipLaunchKernelGGL(k_item_count, dim3(blocks_for(nslots, 256)), dim3(256), 0, st, spt, bprefix,
                       nb, box_sp_off, box_sp, nslots, chunk, counts);
    hipError_t e = scan_exclusive(counts, starts, nslots, nitems, scan_scratch, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_item_fill, dim3(blocks_for(nslots, 256)), dim3(256), 0, st, spt, bprefix,
                       nb, box_sp_off, box_sp, nslots, chunk, (const int *)starts, items);
    hipLaunchKernelGGL(k_set_int, dim3(1), dim3(1), 0, st, queue, 0);
    return hipGetLastError();
}

hipError_t launch_stamp(long long *out, hipStream_t st) {
    hipLaunchKernelGGL(k_stamp, dim3(1), dim3(1), 0, st, out);
    return hipGetLastError();
}

hipError_t launch_set_int(int *p, int v, hipStream_t st) {
    hipLaunchKernelGGL(k_set_int, dim3(1), dim3(1), 0, st, p, v);
    return hipGetLastError();
}

hipError_t launch_zero_ints(int *p, int n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_zero_ints, dim3(blocks_for(n, 256)), dim3(256), 0, st, p, n);
    return hipGetLastError();
}

hipError_t launch_zero_j(const DevFields &f, const DevBox *boxes, const long long *fp, int nb,
                         long long total, hipStream_t st) {
    if (total == 0) return hipSuccess;
    hipLaunchKernelGGL(k_zero_j, dim3(blocks_for(total, 256)), dim3(256), 0, st, f, boxes, fp, nb,
                       total);
    return hipGetLastError();
}

hipError_t launch_fdtd(int prec, const DevFields &f, const DevBox *boxes, const long long *fp,
                       int nb, long long total, hipStream_t st) {
    if (total == 0) return hipSuccess;
    dim3 g(blocks_for(total, 256)), b(256);
    if (prec == 0) {
        hipLaunchKernelGGL(k_faraday<double>, g, b, 0, st, f, boxes, fp, nb, total, 0.5);
        hipLaunchKernelGGL(k_ampere<double>, g, b, 0, st, f, boxes, fp, nb, total);
        hipLaunchKernelGGL(k_faraday<double>, g, b, 0, st, f, boxes, fp, nb, total, 0.5);
    } else {
        hipLaunchKernelGGL(k_faraday<float>, g, b, 0, st, f, boxes, fp, nb, total, 0.5);
        hipLaunchKernelGGL(k_ampere<float>, g, b, 0, st, f, boxes, fp, nb, total);
        hipLaunchKernelGGL(k_faraday<float>, g, b, 0, st, f, boxes, fp, nb, total, 0.5);
    }
    return hipGetLastError();
}

size_t energy_scratch_doubles(int nsp) {
    return (size_t)(2 + nsp) * ENERGY_MAX_GRID;
}

hipError_t launch_energy(int prec, const DevFields &f, const DevBox *boxes, int bi,
                         long long ncells, const EnergySp *sps, int nsp, double *part,
                         double *out, hipStream_t st) {
    if (nsp < 0 || nsp > ENERGY_MAX_SPECIES) return hipErrorInvalidValue;
    EnergyPlan plan;
    plan.nout = 2 + nsp;
    // field partials: slots [0, 2 gf), E and B interleaved
    const unsigned gf = ncells > 0 ? std::min(blocks_for(ncells, 256), (unsigned)ENERGY_MAX_GRID) : 0;
    plan.off[0] = 0; plan.cnt[0] = (int)gf; plan.str[0] = 2;
    plan.off[1] = 1; plan.cnt[1] = (int)gf; plan.str[1] = 2;
    if (gf > 0) {
        if (prec == 0) hipLaunchKernelGGL(k_field_energy<double>, dim3(gf), dim3(256), 0, st, f, boxes, bi, part);
        else hipLaunchKernelGGL(k_field_energy<float>, dim3(gf), dim3(256), 0, st, f, boxes, bi, part);
    }
    // species s: slots [(2 + s) G, (2 + s) G + gs)
    for (int s = 0; s < nsp; ++s) {
        const long long np = sps[s].np;
        const unsigned gs = np > 0 ? std::min(blocks_for(np, 256), (unsigned)ENERGY_MAX_GRID) : 0;
        plan.off[2 + s] = (2 + s) * ENERGY_MAX_GRID;
        plan.cnt[2 + s] = (int)gs;
        plan.str[2 + s] = 1;
        if (gs == 0) continue;
        double *p = part + (size_t)(2 + s) * ENERGY_MAX_GRID;
        if (prec == 0) hipLaunchKernelGGL(k_kinetic_energy<double>, dim3(gs), dim3(256), 0, st, sps[s], p);
        else hipLaunchKernelGGL(k_kinetic_energy<float>, dim3(gs), dim3(256), 0, st, sps[s], p);
    }
    hipLaunchKernelGGL(k_energy_final, dim3(plan.nout), dim3(64), 0, st, (const double *)part, plan, out);
    return hipGetLastError();
}

hipError_t launch_slice_moments(int prec, const DevSpecies *spt, int s, long long np,
                                const DevBox *boxes, double *out, hipStream_t st) {
    if (np == 0) return hipSuccess;
    if (prec == 0)
        hipLaunchKernelGGL(k_slice_moments<0>, dim3(blocks_for(np, 256)), dim3(256), 0, st, spt, s,
                           boxes, out);
    else
        hipLaunchKernelGGL(k_slice_moments<1>, dim3(blocks_for(np, 256)), dim3(256), 0, st, spt, s,
                           boxes, out);
    return hipGetLastError();
}

hipError_t launch_zero_doubles(double *p, long long n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_zero_doubles, dim3(blocks_for(n, 256)), dim3(256), 0, st, p, n);
    return hipGetLastError();
}

hipError_t launch_div_edge(const DevBox *boxes, int bi, long long ncells, double *const v[3],
                           double *out, hipStream_t st) {
    if (ncells == 0) return hipSuccess;
    hipLaunchKernelGGL(k_div_edge, dim3(blocks_for(ncells, 256)), dim3(256), 0, st, boxes, bi,
                       (const double *)v[0], (const double *)v[1], (const double *)v[2], out);
    return hipGetLastError();
}

}  // namespace pic
