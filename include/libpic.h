/*
 * libpic -- MI355X (gfx950) hot path of an explicit electromagnetic
 * particle-in-cell step: shape-factor field gather, relativistic Boris push,
 * charge-conserving (Esirkepov) current deposition and the Yee FDTD update,
 * plus the per-tile particle sort that keeps the LDS-tiled kernels fed.
 *
 * The paper (Sec. II) places its code among explicit-in-time, fully kinetic
 * electromagnetic PIC models and (Sec. III.A) measures it by the rate of
 * particle and cell updates per second; it prints no equation of the step.
 * The operations below are the four parts of such a time step as the
 * published methods define them: B-spline shape factors, the relativistic
 * Boris rotation (Boris 1970), Esirkepov's charge-conserving current
 * deposition (Comput. Phys. Commun. 135, 2001, 144) and Yee's staggered-grid
 * FDTD update (IEEE TAP 14, 1966, 302).  Each entry point names the method
 * it follows.
 *
 * Conventions (every entry point)
 *   - Normalised units: c = eps0 = mu0 = 1.  u = gamma v.
 *   - Particle positions are in CELL units of their box, in [0, n_d).
 *   - Fields of a box are periodic Yee arrays stored x-fastest, index
 *     i + n0*(j + n1*k):  Ex(i+1/2,j,k) Ey(i,j+1/2,k) Ez(i,j,k+1/2),
 *     Bx(i,j+1/2,k+1/2) By(i+1/2,j,k+1/2) Bz(i+1/2,j+1/2,k); J with E.
 *     Several boxes share one allocation per component: box b occupies
 *     cells [cell_base, cell_base + n0*n1*n2).
 *   - dim == 2 is the x-z plane: n[1] == 1, tile[1] == 1, d/dy == 0, all
 *     three velocity and six field components kept.
 *   - Every pointer inside pic_fields / pic_species is a DEVICE pointer
 *     owned by the caller; the library keeps none of them past the call
 *     (except inside a captured step graph, see pic_step).
 *   - All work is enqueued on the stream given to pic_init; calls return
 *     before the GPU finishes.  Host-detectable errors are returned before
 *     any launch; device-side range errors are latched in a flag that
 *     pic_check reports.  Nothing throws across this interface.
 *   - A context is not thread-safe; use one per stream.
 */
#ifndef LIBPIC_H
#define LIBPIC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    PIC_OK = 0,
    PIC_ERR_ARG = 1,     /* bad argument (null pointer, bad size, order, dims) */
    PIC_ERR_CFL = 2,     /* dt above the Courant limit of the box */
    PIC_ERR_OOM = 3,     /* device allocation failed */
    PIC_ERR_DEVICE = 4,  /* a HIP runtime call failed */
    PIC_ERR_RANGE = 5,   /* device flag: a position outside its box, a per-step
                            displacement of 0.999 cell or more, or a
                            non-finite value; such a particle is left in
                            place and deposits nothing */
    PIC_ERR_STATE = 6    /* call order violated (e.g. deposit without a push,
                            tiled kernel before any sort) */
} pic_status;

typedef enum {
    PIC_FP64 = 0,        /* FP64 positions, momenta, weights, fields */
    PIC_FP32_SPLIT = 1   /* int32 cell + FP32 offset positions; FP32 momenta,
                            weights, E and B; FP64 J */
} pic_precision;

typedef enum {
    PIC_KERNEL_DIRECT = 0,  /* one thread per particle, fields and J in global
                               memory (no sort needed) */
    PIC_KERNEL_TILED = 1,   /* one workgroup per (species, tile): E/B staged
                               in LDS, J accumulated in an FP64 LDS tile then
                               flushed with FP64 global atomics (needs
                               pic_sort_tiles).  The staged region carries a
                               1-cell margin on every axis where it fits in
                               LDS (given up on the widest tile edges first),
                               so particles that drifted up to one cell out
                               of their tile since the sort stay on the LDS
                               path; beyond that they use global memory. */
    PIC_KERNEL_BATCHED = 2  /* as TILED, but a persistent grid walks a work
                               queue so uneven tiles and many boxes share one
                               launch: one item per box tile covers every
                               species of the box (one E/B stage, one J flush)
                               unless they hold more than `chunk` particles
                               together, then per-species chunks */
} pic_kernel;

typedef struct {
    int32_t dim;         /* 2 or 3 */
    int32_t n[3];        /* cells per axis, each >= 1 and < 2^20 */
    double dx[3];        /* cell size per axis (> 0) */
    double dt;           /* time step; must satisfy the Courant limit */
    int32_t order;       /* B-spline order 1..3 */
    int32_t tile[3];     /* tile edge per axis for the sort and the tiled
                            kernels (1..16; partial tiles at the high end) */
    int64_t cell_base;   /* offset of this box in the field arrays */
} pic_box_desc;

typedef struct {
    int32_t kernel;      /* pic_kernel */
    int32_t block;       /* threads per workgroup of the tiled kernels
                            (multiple of 64; 64..512 for PIC_FP64, 64..1024
                            for PIC_FP32_SPLIT; 0 = default 256) */
    int32_t chunk;       /* BATCHED: max particles per work item (0 = 4096) */
    int32_t wg_per_cu;   /* BATCHED: persistent workgroups per CU (0 = 2) */
    int32_t lane_stride; /* TILED/BATCHED: lane l of a work item's pass takes
                            particle (l mod G)*stride + l/G, G = ceil(n/stride),
                            so lanes of one wave fall in distinct cells when
                            stride ~ particles per cell (1..64; 0 = 1) */
    int32_t pad;         /* Row padding of the LDS tiles, so that the lanes
                            of one LDS pass (32 for a 4-byte access, 16 for
                            an 8-byte one; a wave sits on a block of tile
                            rows) hit distinct banks.  0: current tile rows,
                            when it fits; 1: field tile rows, then current
                            tile rows, each when it fits; 2: both, giving up
                            margin axes if that is what makes both fit;
                            -1: no padding.  With 16-wide tiles and padded
                            FP32 field rows the library also swaps lane bits
                            4 and 5 of each wave's slots (results are the
                            same; only the lane of a particle changes) */
    int32_t cell_order;  /* Order of the particles inside a tile after
                            pic_sort_tiles.  -1: previous order (tile id
                            only).  1: by class (lx+ly+lz) mod 4 of the
                            tile-local cell (lx,ly,lz), then by the cell
                            lx + tx*(ly + ty*lz), ties stable: cells of one
                            class that share a row differ by a multiple of 4
                            along it, so consecutive particles of different
                            cells never deposit onto one LDS address.  2: as
                            1, then each tile stably split into the whole
                            groups of four of every cell followed by each
                            cell's last (count mod 4) particles, so that
                            aligned groups of four share a cell (the quad
                            pooling of the deposit at lane_stride 1).  3: by
                            the cell lx + tx*(ly + ty*lz) alone, ties stable
                            (restores the cell-major order that lane_stride
                            4 spreads over distinct cells).  4: rank-major:
                            by the rank of a particle among its cell's
                            particles (0..15, ties in cell order), so that
                            consecutive particles of one rank sit in
                            consecutive cells whatever the per-cell counts
                            (for lane_stride 1).  1..4 apply when tile id
                            and cell fit a 31-bit key.
                            0 = default: 2 for BATCHED, else -1.  The DPP
                            quad pooling of the deposit runs only with
                            lane_stride 1 and order 2. */
    int32_t quad_spread; /* TILED/BATCHED at lane_stride 1: 1 = the 16 quads
                            of a wave are taken ceil(nquads/16) quads apart
                            in a species' tile range instead of in a row, so
                            cells holding several quads of particles spread
                            over waves; -1 = in a row; 0 = default: 1 for a
                            species with at least 6 particles per cell of its
                            box on average, else -1. */
    int32_t margin;      /* TILED/BATCHED: 0 = stage the 1-cell margin on the
                            axes where it fits (default); -1 = no margin
                            (particles out of their tile since the sort take
                            the global path; smaller LDS stage). */
    int32_t pusher;      /* 0 = relativistic Boris (default); 1 = the pusher
                            of Vay (Phys. Plasmas 15, 056701, 2008), exact
                            for the E x B drift at any speed */
    int32_t gather;      /* 0 = every field component gathered with order-n
                            shapes on all axes (default); 1 = Galerkin form:
                            order n - 1 along each axis on which the
                            component sits at half-integer points (order 0 =
                            the nearest node) */
} pic_tuning;

typedef struct {
    void *E[3];          /* FP64 (PIC_FP64) or FP32 (PIC_FP32_SPLIT) */
    void *B[3];
    double *J[3];        /* FP64 in both precisions */
} pic_fields;

typedef struct {
    int64_t np;          /* particles (0 allowed; < 2^31) */
    double q, m;         /* charge and mass of one physical particle */
    int32_t box;         /* index into the box list given to pic_init */
    double *x[3];        /* PIC_FP64: positions; x[1] unused in 2D */
    int32_t *cell;       /* PIC_FP32_SPLIT: linear cell id within the box */
    float *off[3];       /* PIC_FP32_SPLIT: in-cell offsets in [0, 1);
                            off[1] unused in 2D */
    void *u[3];          /* momenta, FP64 or FP32 per precision */
    void *w;             /* weights, FP64 or FP32 per precision */
} pic_species;

typedef struct pic_ctx pic_ctx;

/* Create a context for nboxes boxes at the given precision, bound to
 * `stream` (a hipStream_t; NULL = the null stream).  Validates every box
 * (dims, order, tile, Courant limit dt <= 1/sqrt(sum 1/dx_d^2) over the
 * box's axes) and allocates the context's own scratch (device error flag,
 * tile tables).  `tuning` may be NULL (defaults: BATCHED for FP32_SPLIT,
 * TILED for FP64).  On error *ctx is NULL. */
pic_status pic_init(pic_ctx **ctx, const pic_box_desc *boxes, int32_t nboxes,
                    pic_precision prec, void *stream, const pic_tuning *tuning);

/* Per-tile stable counting sort.  The paper is silent on particle ordering;
 * this is the library's own data structure: it groups particles by the tile
 * of their cell so the tiled kernels can stage each tile's E/B and J in LDS.
 * Least-significant-digit radix passes over the tile id permute every
 * species' particle arrays IN PLACE so that particles are grouped by tile
 * id = tx + ntx*(ty + nty*tz) of their cell, ties kept in their previous
 * order (with pic_tuning.cell_order, ordered by cell inside each tile first);
 * particles with an invalid position go to a bucket after the last tile.
 * The per-tile offsets are kept in the context for the tiled kernels.
 * Optional outputs, each an array of nsp device pointers (the array itself
 * on the host; it or any entry may be NULL; each entry owned by the caller,
 * np ints, or ntiles+1 for offsets): perm_out[s][i] = previous index of the
 * particle now at i; key_out[s][i] = its tile id; tile_offset_out[s] =
 * ntiles+1 exclusive offsets.  Species must be passed in the same order to
 * every call.  Errors: PIC_ERR_ARG (bad species table), PIC_ERR_STATE
 * (between pic_gather_push and pic_deposit_J), PIC_ERR_OOM (scratch). */
pic_status pic_sort_tiles(pic_ctx *ctx, const pic_species *sp, int32_t nsp,
                          int32_t *const *perm_out, int32_t *const *key_out,
                          int32_t *const *tile_offset_out);

/* Field gather and particle push.  Gather: E, B at x^n as the sum over the
 * Yee points of each component of the field value times the product of
 * order-n B-spline shape factors along the three axes (the same order on
 * every stagger).  Push: the relativistic Boris rotation (Boris 1970)
 * u^(n-1/2) -> u^(n+1/2) with h = q dt / (2 m): half electric kick, magnetic
 * rotation by t = h B / gamma-, half electric kick; then the advance
 * x^(n+1) = x^n + dt u^(n+1/2) / (gamma^(n+1/2) dx_d) per axis.  Both are
 * the particle half of the explicit PIC step the paper names (Sec. II).
 * x^n is kept in context scratch for pic_deposit_J.  Until that call FP64
 * positions are left unwrapped (within one cell outside [0, n)); split
 * positions are stored wrapped, their cell change kept in scratch.
 * A particle with |dx| >= 0.999 cell or a non-finite value is left in place
 * and latches PIC_ERR_RANGE for pic_check.  Tiled/batched forms need a
 * preceding pic_sort_tiles (else PIC_ERR_STATE). */
pic_status pic_gather_push(pic_ctx *ctx, const pic_fields *f, pic_species *sp,
                           int32_t nsp);

/* Charge-conserving current deposition of Esirkepov (Comput. Phys. Commun.
 * 135, 2001, 144): zero J of every box, then for each particle the move
 * x^n -> x^(n+1) recorded by the last pic_gather_push is deposited as
 * W^x = dSx (S0y S0z + dSy S0z / 2 + S0y dSz / 2 + dSy dSz / 3) (and
 * cyclically), J_x = -(q w dx / (dt dV)) times the running sum of W^x along
 * x, so that the discrete continuity equation d(rho)/dt + div J = 0 holds
 * to rounding.  Then positions are wrapped periodically.  J is FP64 in both
 * precisions, accumulated with atomics (order of the sum unspecified).  In
 * the tiled and batched split form each work item first sums its
 * contributions in LDS as 64-bit fixed point (each FP32 contribution scaled
 * by a power of two chosen from the item's largest |q w dx / (dt dV)| and
 * truncated at 2^-30 of it; exact, order-independent sums), then adds them
 * to J in FP64; a non-finite weight latches PIC_ERR_RANGE there.
 * PIC_ERR_STATE without a preceding pic_gather_push on the same species. */
pic_status pic_deposit_J(pic_ctx *ctx, pic_fields *f, pic_species *sp,
                         int32_t nsp);

/* Fused form of pic_gather_push + pic_deposit_J in one kernel pass:
 * zero J, then gather, push, advance, deposit, wrap. */
pic_status pic_advance(pic_ctx *ctx, pic_fields *f, pic_species *sp,
                       int32_t nsp);

/* Yee's staggered-grid FDTD update (IEEE TAP 14, 1966, 302), periodic, of
 * every box: B -= (dt/2) curl E; E += dt (curl B - J); B -= (dt/2) curl E,
 * with the curls taken as one-cell differences on the Yee stagger (2D: no
 * d/dy terms), so E and B are co-timed at integer steps for the next gather.
 * The field half of the explicit EM step the paper names (Sec. II).
 * E, B in the context's precision, J FP64; all arrays owned by the caller. */
pic_status pic_fdtd_step(pic_ctx *ctx, pic_fields *f);

/* One whole step (optional sort, pic_advance, pic_fdtd_step) recorded once
 * into a HIP graph per distinct (fields, species, sort) binding and
 * replayed with a single graph launch afterwards.  The caller must keep the
 * bound arrays alive while the context may replay the graph. */
pic_status pic_step(pic_ctx *ctx, pic_fields *f, pic_species *sp, int32_t nsp,
                    int32_t sort);

/* Charge density rho = sum q w S S S / dV on the nodes of box `box`, FP64,
 * ADDED into rho (ncells of that box).  A check, not part of the step. */
pic_status pic_deposit_rho(pic_ctx *ctx, const pic_species *sp, int32_t nsp,
                           int32_t box, double *rho);

/* Node divergence of an E-staggered vector field (J or E, FP64) of box
 * `box` into out (ncells).  A check, not part of the step. */
pic_status pic_div_edge(pic_ctx *ctx, int32_t box, double *const v[3],
                        double *out);

/* Energies of box `box`, a check beside the step, not part of it: the
 * electromagnetic field energy and the relativistic kinetic energy
 * m (gamma - 1) c^2 of the particles of the fully kinetic model (Sec. II),
 * whose sum the explicit scheme keeps up to its truncation error.  FP64
 * sums on the device into out (a DEVICE array of 2 + nsp doubles owned by
 * the caller, overwritten):
 *   out[0] = 1/2 sum over cells of E.E dV,  out[1] = 1/2 sum of B.B dV
 *            (eps0 = mu0 = 1; each component at its own Yee point);
 *   out[2 + s] = sum over the particles of species s of w m (gamma - 1),
 *            gamma - 1 evaluated as u.u / (1 + gamma); 0 for a species of
 *            another box.
 * Deterministic: per-workgroup partial sums (in context scratch, allocated
 * on first use) are added in a fixed order.  At most 16 species.
 * Errors: PIC_ERR_ARG (bad box, NULL out or field pointer, bad species,
 * nsp > 16), PIC_ERR_OOM (scratch). */
pic_status pic_energy(pic_ctx *ctx, const pic_fields *f, const pic_species *sp,
                      int32_t nsp, int32_t box, double *out);

/* pic_energy for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving or diagnostics loops, harnesses that forbid
 * hipMalloc.  Same arguments, results and errors as pic_energy (bit-equal:
 * the same kernels and summation order), but it allocates nothing: its
 * partial sums live in a fixed 144 KiB device array of the library, one copy
 * per GPU, looked up once by pic_init and held until the process ends.  The
 * array bounds the call to at most 16 species (PIC_ERR_ARG beyond; the cell
 * and particle counts are not bounded).  Every call on one GPU shares that
 * GPU's array, and each call overwrites the slots it reads: calls that
 * overlap in time on one GPU (several streams or threads) race and must be
 * ordered by the caller. */
pic_status pic_energy_noalloc(pic_ctx *ctx, const pic_fields *f, const pic_species *sp,
                              int32_t nsp, int32_t box, double *out);

/* Decomposition of one periodic box into slabs along z, the boxes of this
 * context: the domain decomposition of the paper's multi-GPU runs (Sec.
 * III.B, Fig. 2), held on one GPU.  Box s of the context is slab s (z
 * order, periodic neighbours): it owns global layers [z0_s, z0_s + nz_s)
 * and stores them at local z in [guard, guard + nz_s), with `guard` layers
 * below and above; n[2] of box s = nz_s + 2 guard.  All slabs share dim,
 * nx, ny, dx, dt and order; guard >= 3 (the Yee update and the widest
 * order-3 stencils stay valid with 3) and nz_s >= 2 guard
 * (PIC_ERR_ARG otherwise).  Particles live in the interiors; field and
 * particle arrays are the caller's, as for any box.  One step is:
 *   pic_slab_fill_guards; [pic_sort_tiles]; pic_advance (all slabs in one
 *   launch); pic_slab_reduce_j; pic_fdtd_step; pic_slab_migrate; and a
 *   pic_sort_tiles before the next tiled particle update whenever counts
 *   changed.
 * Results equal those of the undivided box up to the order of the J sums.
 *
 * pic_slab_fill_guards: E and B guard layers <- the owning neighbour's
 * interior layers (before the gather). */
pic_status pic_slab_fill_guards(pic_ctx *ctx, pic_fields *f, int32_t guard);

/* pic_slab_reduce_j: every guard layer's J is added to the neighbour
 * interior layer it covers (pulled by the interior, deterministic), then
 * the complete interior J is copied back into the guards (after the
 * deposit, before the Yee update). */
pic_status pic_slab_reduce_j(pic_ctx *ctx, pic_fields *f, int32_t guard);

/* pic_slab_migrate: particles whose position left their slab's interior
 * (they are at most one cell into a guard) move to the neighbour slab's
 * arrays, z shifted into its frame.  sp: nsp = nslab x kinds species given
 * slab-major (sp[i].box == i / kinds; kind k of every slab is one particle
 * kind), each with its current count np; cap[i] (host) = capacity of its
 * arrays in particles.  Each species keeps its stayers in order, then the
 * arrivals from the slab below, then from above.  np_out[i] (host) gets the
 * new counts; the call waits for the stream once (to learn the counts).
 * PIC_ERR_ARG if a count would exceed its capacity (nothing is changed). */
pic_status pic_slab_migrate(pic_ctx *ctx, pic_species *sp, int32_t nsp, int32_t guard,
                            const int64_t *cap, int64_t *np_out);

/* ---- Laser-plasma boundaries (the steps around the periodic core of a
 * laser-wakefield run, paper Abstract and Sec. III.A: a laser enters from an
 * antenna, the fields are absorbed at the ends of z, and the frame moves
 * with the laser).  z is the laser axis; x and y stay periodic. */

/* Absorbing layers of `cells` cells at both ends of z of box `box` (in the
 * frame of the moving window, see pic_window_shift): Maxwell's equations
 * with an electric and an equal magnetic conductivity sigma(d) = sigma_max
 * (d / cells)^power at depth d into a layer, which match the vacuum
 * impedance, so a wave at normal incidence enters without reflection in
 * the continuum limit and decays as exp(-integral sigma dz).  pic_fdtd_step
 * then integrates the decay of each sub-step exactly: F <- exp(-sigma tau) F
 * + (1 - exp(-sigma tau)) / sigma * (curl source), sigma at each component's
 * own Yee point.  cells = 0 removes the layers.  PIC_ERR_ARG unless
 * 0 <= 2 cells <= n_z, sigma_max >= 0, 0 <= power <= 8.  Waits for the
 * stream (set-up call). */
pic_status pic_set_absorber(pic_ctx *ctx, int32_t box, int32_t cells, double sigma_max,
                            int32_t power);

/* Laser antenna: a current sheet at the E_x points of cell layer k of the
 * window frame, K_x(x, y, t) = -2 E0 exp(-r^2 / waist^2) exp(-((t - t0) /
 * tau)^2) sin(omega (t - t0)), r from (x0, y0) (cell units times dx); a
 * current sheet K radiates E = -K / 2 on both sides, so each emitted wave
 * has amplitude E0 (the backward one is for the absorbing layer).  Added
 * as K / dz into J_x of that layer: call after pic_deposit_J (or
 * pic_advance) and before pic_fdtd_step, with t = the time of that J
 * (t^(n+1/2) = (n + 1/2) dt). */
typedef struct {
    int32_t k;           /* window-frame cell layer of the sheet */
    double E0;           /* emitted field amplitude */
    double omega;        /* angular frequency */
    double waist;        /* 1/e field radius */
    double x0, y0;       /* centre of the spot */
    double t0, tau;      /* centre and 1/e half-length of the envelope */
} pic_antenna;
pic_status pic_antenna_add(pic_ctx *ctx, pic_fields *f, int32_t box, const pic_antenna *an,
                           double t);

/* Moving window: the frame of box `box` advances one cell along +z.  The
 * field arrays are circular in z: the frame's layer 0 sits at array layer
 * zoff (pic_window_offset), and a shift zeroes E and B of the array layer
 * that leaves the frame's bottom (it becomes the new top layer), removes
 * the particles in it (the others keep their order) and advances zoff by
 * one; no field data moves.  inject[i] (species i of the box) are new
 * particles for the new top layer, positions in the window frame (FP64: z
 * in [n_z - 1, n_z); split: cell ids of that layer), appended after the
 * kept ones (np 0 for none; same precision and arrays as sp[i]).  cap[i]
 * (host) = capacity of sp[i]'s arrays; np_out[i] (host) = the new counts
 * (species of other boxes unchanged).  Waits for the stream to learn the
 * counts; PIC_ERR_ARG if a count would exceed its capacity.  Positions
 * of all particles stay in array coordinates, so the particle kernels need
 * no change; a pic_sort_tiles must precede the next tiled update. */
pic_status pic_window_shift(pic_ctx *ctx, pic_fields *f, pic_species *sp, int32_t nsp,
                            int32_t box, const pic_species *inject, const int64_t *cap,
                            int64_t *np_out);

/* Array layer of the window frame's layer 0 of box `box`. */
pic_status pic_window_offset(pic_ctx *ctx, int32_t box, int32_t *zoff);

/* ---- Electrostatic variant (the paper's codes include an electrostatic
 * PIC solver beside the electromagnetic one, Sec. II and IV).  One ES step
 * is pic_es_solve then pic_es_push; B is not used.
 *
 * pic_es_solve: charge density rho of the species of box `box` (as
 * pic_deposit_rho), its mean removed (a neutralising background), the
 * discrete periodic Poisson equation -div grad phi = rho - <rho> solved by
 * conjugate gradients from phi = 0 with the 7-point Yee Laplacian (5-point
 * in 2D) until |r| <= tol |rho - <rho>| (checked every 16 iterations), the
 * mean of phi removed, and E = -grad phi written at the Yee E points
 * (E_x(i+1/2) = -(phi(i+1) - phi(i)) / dx ...) into f->E of the box, so
 * div E = rho - <rho> to the tolerance.  phi: DEVICE array of the box's
 * ncells doubles (caller-owned, overwritten).  *iters_out / *res_out (host,
 * may be NULL): iterations and final relative residual.  Waits for the
 * stream every 16 iterations.  PIC_ERR_STATE if max_iter is reached first
 * (E is still written). */
pic_status pic_es_solve(pic_ctx *ctx, const pic_species *sp, int32_t nsp, int32_t box,
                        pic_fields *f, double *phi, double tol, int32_t max_iter,
                        int32_t *iters_out, double *res_out);

/* pic_es_push: every particle gathers E at x^n (order-n shapes on each
 * component's Yee points, as pic_gather_push), takes the Boris step with
 * B = 0 (u += q E dt / m), advances x^(n+1) = x^n + dt u / (gamma dx) and
 * wraps; no current.  One thread per particle (no sort needed; a later
 * tiled call needs pic_sort_tiles again). */
pic_status pic_es_push(pic_ctx *ctx, const pic_fields *f, pic_species *sp, int32_t nsp);

/* In-situ reduction (a diagnostic beside the step, the kind of streaming
 * analysis the paper's codes run in place of full output, Sec. IV):
 * per-layer moments along z of every species of box `box`, in the frame of
 * the moving window (layer (k - zoff) mod n_z of array layer k):
 * out[(s n_z + k) 5 + q], q = 0 sum w, 1..3 sum w u_d, 4 sum w m (gamma - 1)
 * (gamma - 1 = u.u / (1 + gamma)).  out: DEVICE array of 5 n_z nsp doubles
 * (caller-owned, overwritten; zero for species of other boxes).  FP64
 * atomics (summation order unspecified). */
pic_status pic_slice_moments(pic_ctx *ctx, const pic_species *sp, int32_t nsp, int32_t box,
                             double *out);

/* Wait for the stream and report the first device-side error (then clear). */
pic_status pic_check(pic_ctx *ctx);

/* Release the context and its scratch (waits for the stream). NULL is OK. */
pic_status pic_free(pic_ctx *ctx);

/* Static text for a status; and the message of the last failed call. */
const char *pic_status_str(pic_status s);
const char *pic_last_error(void);

/* Number of workgroups the context's kernels fill the device with (CUs). */
int32_t pic_device_cus(pic_ctx *ctx);

/* Timing of the tiled particle kernels (TILED/BATCHED forms).  With on != 0
 * every later launch of the tiled kernel and the straggler kernel that
 * follows it -- by pic_advance, pic_gather_push, pic_deposit_J, or inside
 * the graph of pic_step (graphs are recorded separately with and without
 * timing) -- is bracketed by two one-thread kernels on the context's stream
 * that store the device's constant-rate wall clock (HIP events recorded
 * inside a graph give no elapsed time on this runtime).  pic_kernel_ms
 * waits for the stream and returns in *ms the time between the two stamps
 * of the most recent timed launch (both kernels plus the launch gaps, a few
 * microseconds each); PIC_ERR_STATE if none was recorded since
 * pic_set_timing. */
pic_status pic_set_timing(pic_ctx *ctx, int32_t on);
pic_status pic_kernel_ms(pic_ctx *ctx, float *ms);

#ifdef __cplusplus
}
#endif

#endif
