/*
 * Plain FP64 CPU oracle of one explicit electromagnetic particle-in-cell step.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library calls, links or
 * includes this file; only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark load it.  It shares no code, header, table
 * or helper with the GPU library.
 *
 * What it follows.  The paper (Sec. II: an explicit, fully kinetic
 * electromagnetic PIC model; Sec. IV: the time-based EM code) names the
 * method but prints no equation of it, so each function below is the
 * textbook definition of the published method the step is built from:
 *   - B-spline particle shape factors of order 1..3;
 *   - the relativistic Boris rotation (Boris 1970);
 *   - the charge-conserving current deposition of Esirkepov
 *     (Comput. Phys. Commun. 135 (2001) 144);
 *   - the staggered-grid FDTD Maxwell solver of Yee (IEEE TAP 14 (1966) 302).
 * Where these leave a choice open (units, stagger, time levels, wrap rule)
 * the reading is stated at the function.
 *
 * Conventions (normalised units): c = eps0 = mu0 = 1.  Particle positions are
 * stored in CELL units, xi_d = x_d / dx_d, inside [0, n_d).  Momentum per
 * unit mass u = gamma v.  Fields live on a periodic Yee grid stored x-fastest,
 * index i + n0*(j + n1*k):
 *   Ex (i+1/2, j, k)   Ey (i, j+1/2, k)   Ez (i, j, k+1/2)
 *   Bx (i, j+1/2, k+1/2) By (i+1/2, j, k+1/2) Bz (i+1/2, j+1/2, k)
 *   J co-located with E, charge density rho on nodes (i, j, k).
 * dim == 2 means the x-z plane (n[1] must be 1, d/dy == 0, all 3 velocity
 * and all 6 field components kept).
 *
 * Parity status: every function here is pinned by the CPU test-suite against
 * closed forms, invariants, special cases or brute force; none is
 * "parity unpinned".
 */
#ifndef PIC_ORACLE_H
#define PIC_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int32_t dim;      /* 2 (x-z plane) or 3 */
    int32_t n[3];     /* cells per axis (n[1] == 1 when dim == 2) */
    double dx[3];     /* cell size per axis */
    double dt;        /* time step */
    int32_t order;    /* B-spline order, 1..3 */
} orc_grid;

typedef struct {
    int64_t np;       /* number of macro-particles */
    double q, m;      /* charge and mass of one physical particle */
    double *x[3];     /* positions in cell units; x[1] ignored when dim == 2 */
    double *u[3];     /* u = gamma v (c = 1) */
    double *w;        /* macro-particle weight (physical particles per macro) */
} orc_species;

/* B-spline of the given order evaluated at distance a (any sign). */
double orc_shape(int32_t order, double a);

/* Field values seen by one particle at position xi (cell units). */
void orc_gather(const orc_grid *g, double *const E[3], double *const B[3],
                const double xi[3], double Ep[3], double Bp[3]);

/* One relativistic Boris step of u (in place), charge-to-mass q/m. */
void orc_boris(double q, double m, double dt, const double Ep[3],
               const double Bp[3], double u[3]);

/* Esirkepov current of one particle moving x0 -> x1 (unwrapped, cell units),
 * ADDED into J.  vy is the out-of-plane velocity, used only when dim == 2. */
void orc_deposit(const orc_grid *g, double *J[3], double q, double w,
                 const double x0[3], const double x1[3], double vy);

/* Yee updates on the periodic grid. */
void orc_faraday(const orc_grid *g, double *const E[3], double *B[3], double h);
void orc_ampere(const orc_grid *g, double *E[3], double *const B[3],
                double *const J[3], double dt);
/* B half step, E full step, B half step. */
void orc_fdtd_step(const orc_grid *g, double *E[3], double *B[3],
                   double *const J[3]);

/* Periodic wrap of one coordinate after the deposit. */
double orc_wrap(double x, double L);

/* Particle part of one step for every species: J is zeroed, then for each
 * particle in index order: gather at x^n, Boris push, advance, deposit,
 * wrap. */
void orc_particles_step(const orc_grid *g, double *const E[3],
                        double *const B[3], double *J[3],
                        orc_species *sp, int32_t nsp);

/* Whole step: particles, then the Yee update. */
void orc_pic_step(const orc_grid *g, double *E[3], double *B[3], double *J[3],
                  orc_species *sp, int32_t nsp);

/* Charge density on nodes (ADDED into rho). */
void orc_rho(const orc_grid *g, double *rho, const orc_species *sp);

/* Discrete divergence of J on nodes. */
void orc_div_j(const orc_grid *g, double *const J[3], double *divj);

/* Field energy 1/2 sum(E^2+B^2) dV and kinetic energy sum w m (gamma-1). */
double orc_field_energy(const orc_grid *g, double *const E[3],
                        double *const B[3]);
double orc_kinetic_energy(const orc_species *sp);

/* Absorbing layers of `cells` cells at both z ends with equal electric and
 * magnetic conductivity sigma(d) = sigma_max (d / cells)^power at depth d. */
typedef struct {
    int32_t cells;
    double sigma_max;
    int32_t power;
} orc_absorber;

/* Conductivity at height z (cell units) of a box nz cells long. */
double orc_absorber_sigma(const orc_absorber *a, double z, double nz);

/* Yee step (B half, E full, B half) with the absorbing layers; each
 * sub-step integrates the conductive decay exactly.  The layers sit at the
 * window-frame ends: a component at array height z has frame height
 * (z - zoff) mod nz (zoff = 0 without a moving window). */
void orc_fdtd_step_absorb(const orc_grid *g, double *E[3], double *B[3], double *const J[3],
                          const orc_absorber *a, double zoff);

/* Laser antenna: a current sheet at the E_x points of cell layer k. */
typedef struct {
    int32_t k;        /* cell layer of the sheet */
    double E0;        /* emitted field amplitude */
    double omega;     /* angular frequency */
    double waist;     /* 1/e field radius */
    double x0, y0;    /* centre */
    double t0, tau;   /* centre and 1/e half-length of the envelope in time */
} orc_antenna;

/* Adds the antenna's current at time t into J[0]. */
void orc_antenna_add(const orc_grid *g, double *J[3], const orc_antenna *an, double t);

/* Moving window by one cell along +z: fields shift toward -z with a zero
 * top layer; particles shift and those leaving are removed (order kept). */
void orc_window_shift_fields(const orc_grid *g, double *E[3], double *B[3]);
int64_t orc_window_shift_particles(const orc_grid *g, orc_species *sp);

/* Electrostatic variant: E = -grad phi at the Yee E points; the particle
 * update in E alone (gather, Boris with B = 0, advance, wrap; no deposit). */
void orc_es_field(const orc_grid *g, const double *phi, double *E[3]);
void orc_es_particles_step(const orc_grid *g, double *const E[3], orc_species *sp, int32_t nsp);

/* Variants: the relativistic pusher of Vay (2008); the Galerkin gather
 * (order lowered by one along each axis where the component is at
 * half-integer points; order 0 = nearest node); the particle step with
 * pusher (0 Boris, 1 Vay) and gather (0 default, 1 Galerkin) chosen. */
void orc_vay(double q, double m, double dt, const double Ep[3], const double Bp[3], double u[3]);
void orc_gather_galerkin(const orc_grid *g, double *const E[3], double *const B[3],
                         const double xi[3], double Ep[3], double Bp[3]);
void orc_particles_step_opts(const orc_grid *g, double *const E[3], double *const B[3],
                             double *J[3], orc_species *sp, int32_t nsp, int32_t pusher,
                             int32_t gather);

/* Per-layer moments along z (window frame, zoff as the moving window):
 * out[5 k + q] += sum over the layer's particles of w, w u_x, w u_y, w u_z,
 * w m (gamma - 1). */
void orc_slice_moments(const orc_grid *g, const orc_species *sp, int32_t zoff, double *out);

/* Rank-major order inside each tile of a (tile, cell) key: by rank of a
 * particle within its cell (capped at 2^rbits - 1), ties in cell order.  A
 * layout choice of the GPU sort (pic_tuning.cell_order 4). */
void orc_rank_major(int64_t np, const int64_t *key, int32_t cbits, int32_t rbits, int32_t *perm);

/* Tile id of every particle, tile = cell / tile[d] per axis (partial tiles at
 * the high end allowed), id = tx + ntx*(ty + nty*tz). */
void orc_tile_keys(const orc_grid *g, const int32_t tile[3],
                   const orc_species *sp, int32_t *key);

/* Stable sort of particle indices by key (ties kept in index order), with
 * per-key counts and exclusive offsets (nkeys+1 entries). */
void orc_stable_sort(int64_t np, const int32_t *key, int32_t nkeys,
                     int32_t *perm, int32_t *count, int32_t *offset);

/* Within-tile cell order of the tiled sort: for the particle's cell with
 * tile-local coordinates (lx, ly, lz) (ly = 0 in 2D), key = tile id
 * << (cbits + 2) | ((lx + ly + lz) mod 4) << cbits | (lx + tile[0]*(ly +
 * t1*lz)), t1 = tile[1] in 3D and 1 in 2D.  A layout choice of the GPU
 * sort, not part of the method: sorting by it groups a tile's particles by
 * cell class, then cell. */
void orc_cell_order_keys(const orc_grid *g, const int32_t tile[3], int32_t cbits,
                         const orc_species *sp, int64_t *key);

/* Cell order without classes: key = tile id << cbits | (lx + tile[0]*(ly +
 * t1*lz)), the same tile-local cell index as orc_cell_order_keys. */
void orc_tile_cell_keys(const orc_grid *g, const int32_t tile[3], int32_t cbits,
                        const orc_species *sp, int64_t *key);

/* Stable sort of particle indices by a 64-bit key (ties in index order). */
void orc_stable_perm(int64_t np, const int64_t *key, int32_t *perm);

/* The cell order followed by a stable split of every tile (tile id = key >>
 * (cbits + 2)): first, in sorted order, the particles of each cell's whole
 * groups of four (the first count - count mod 4 of its run), then the
 * remaining count mod 4 of every cell, also in sorted order.  Also a layout
 * choice of the GPU sort. */
void orc_quad_order(int64_t np, const int64_t *key, int32_t cbits, int32_t *perm);

#ifdef __cplusplus
}
#endif

#endif
