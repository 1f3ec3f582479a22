// Device-side descriptors of libpic (boxes, species, fields, launch
// parameters) and the declarations of the kernel launchers.  Internal to the
// library; the public interface is include/libpic.h.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pic {

struct DevBox {
    int dim;            // 2 or 3
    int order;
    int n[3];
    int tile[3];
    int nt[3];          // tiles per axis
    int ntiles;
    int small;          // 1 if some n[d] is below the widest stencil (needs
                        // general modulo wrapping)
    long long cell_base;
    long long ncells;
    double dt;
    double dx[3];
    double inv_nx, inv_nxy;   // 1/n[0], 1/(n[0] n[1]) for index decoding
    // absorbing layers of abs_cells cells at both z ends of the window
    // frame, conductivity abs_sigma (d / abs_cells)^abs_power at depth d
    // (abs_cells == 0: none); zoff: array layer of the window frame's
    // layer 0 (a moving window advances it; the arrays are circular in z)
    int abs_cells, abs_power;
    double abs_sigma;
    int zoff;
};

struct DevSpecies {
    long long np;
    double q, m;
    int box;
    int tile_base;      // first (species, tile) slot of this species
    double *x[3];
    int *cell;
    float *off[3];
    void *u[3];
    void *w;
    // scratch of the split push/deposit: x^n
    double *xo[3];
    int *cello;
    float *offo[3];
    int *carry;         // split: cell change per axis, 2 bits each (+1)
    int *strag;         // tiled kernels: particles outside tile + margin
    // exclusive per-tile offsets from the last sort, ntiles+2 entries
    // (the extra bucket holds particles with invalid positions)
    int *tile_off;
    int pusher;         // 0 Boris, 1 Vay
    int galerkin;       // 1: Galerkin gather (order - 1 along staggered axes)
    int spread;         // tiled kernels at lane stride 1: a wave's 16 quads
                        // are taken ceil(nquads/16) quads apart, not in a
                        // row (several quads per cell)
};

struct DevFields {
    void *E[3];
    void *B[3];
    double *J[3];
};

// Work item of the batched kernel.  s >= 0: particles [p0, p1) of species s
// in tile t.  s < 0: every particle of every species of box -1 - s in tile t
// (p0, p1 unused), one field stage and one current flush for all of them.
// t < 0 marks the end of the queue.
struct Item {
    int s, t, p0, p1;
};

enum Mode { MODE_PUSH = 1, MODE_DEPOSIT = 2, MODE_FUSED = 3 };

struct KParams {
    const DevBox *boxes;
    const DevSpecies *species;
    int nsp;
    DevFields f;
    int *err;                 // device error flag (bit 0: range)
    // TILED: block b -> species via prefix of tiles (nsp+1 entries)
    const int *sp_tile_prefix;
    // BATCHED: persistent queue of items
    const Item *items;
    const int *nitems;
    int *queue;
    int lds_field_bytes;      // offset of the J region in dynamic LDS
    int lane_stride;          // lane -> particle stride inside a work item
    int quad;                 // 1: fused kernels pool the deposit of aligned quads
    int margin[3];            // cells staged around each tile per axis (0 or 1)
    int jrow;                 // minimum row length of the LDS current tile
    int frow;                 // minimum row length of the LDS field tile
    int falign;               // 1: field rows from and to multiples of 16
                              // bytes (stage copied 16 bytes a lane)
    int lane_swz;             // 1: slots of a wave swap lane bits 4 and 5, so
                              // that with 16-wide tile rows the 32 lanes of
                              // one LDS pass of a 4-byte field read hold
                              // rows r and r + 2 (see frow)
    int *strag_count;         // per species: entries in its straggler list
    // species of each box (CSR: box_sp[box_sp_off[b] .. box_sp_off[b+1]))
    const int *box_sp_off;
    const int *box_sp;
};

}  // namespace pic
