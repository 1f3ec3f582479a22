/*
 * Plain FP64 CPU oracle of one explicit electromagnetic PIC step.
 * TEST INFRASTRUCTURE ONLY -- see pic_oracle.h for scope, conventions and the
 * published methods each function follows.  Written for readability, not
 * speed: every sum is a plain loop in particle-index order.
 */
#include "pic_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ---------------------------------------------------------------- shapes */

/* Centred cardinal B-spline of order 1, 2, 3 (the box function convolved
 * with itself order times), support |a| < (order+1)/2. */
double orc_shape(int32_t order, double a)
{
    a = fabs(a);
    if (order == 1) {
        return a < 1.0 ? 1.0 - a : 0.0;
    }
    if (order == 2) {
        if (a <= 0.5) return 0.75 - a * a;
        if (a < 1.5) return 0.5 * (1.5 - a) * (1.5 - a);
        return 0.0;
    }
    if (order == 3) {
        if (a < 1.0) return (4.0 - 6.0 * a * a + 3.0 * a * a * a) / 6.0;
        if (a < 2.0) return (2.0 - a) * (2.0 - a) * (2.0 - a) / 6.0;
        return 0.0;
    }
    return 0.0;
}

static int64_t wrapi(int64_t i, int64_t n)
{
    int64_t r = i % n;
    return r < 0 ? r + n : r;
}

static int64_t cell_index(const orc_grid *g, int64_t i, int64_t j, int64_t k)
{
    return wrapi(i, g->n[0]) + (int64_t)g->n[0] *
           (wrapi(j, g->n[1]) + (int64_t)g->n[1] * wrapi(k, g->n[2]));
}

/* Lowest node whose shape can be non-zero for a particle at xi, on nodes
 * placed at i + stagger: every node with |xi - i - stagger| < (order+1)/2. */
static int64_t window_lo(int32_t order, double xi, double stagger)
{
    return (int64_t)floor(xi - stagger - 0.5 * (order + 1));
}

/* ---------------------------------------------------------------- gather */

/* Each component is interpolated from its own staggered points with the
 * same order in every direction ("energy-conserving" gather). */
static double gather_one(const orc_grid *g, const double *F, const double xi[3],
                         const double st[3])
{
    const int32_t o = g->order;
    double sum = 0.0;
    int64_t lo[3];
    for (int d = 0; d < 3; ++d) lo[d] = window_lo(o, xi[d], st[d]);
    if (g->dim == 2) {
        for (int64_t k = lo[2]; k <= lo[2] + o + 2; ++k) {
            double sz = orc_shape(o, xi[2] - ((double)k + st[2]));
            for (int64_t i = lo[0]; i <= lo[0] + o + 2; ++i) {
                double sx = orc_shape(o, xi[0] - ((double)i + st[0]));
                sum += F[cell_index(g, i, 0, k)] * sx * sz;
            }
        }
        return sum;
    }
    for (int64_t k = lo[2]; k <= lo[2] + o + 2; ++k) {
        double sz = orc_shape(o, xi[2] - ((double)k + st[2]));
        for (int64_t j = lo[1]; j <= lo[1] + o + 2; ++j) {
            double sy = orc_shape(o, xi[1] - ((double)j + st[1]));
            for (int64_t i = lo[0]; i <= lo[0] + o + 2; ++i) {
                double sx = orc_shape(o, xi[0] - ((double)i + st[0]));
                sum += F[cell_index(g, i, j, k)] * sx * sy * sz;
            }
        }
    }
    return sum;
}

void orc_gather(const orc_grid *g, double *const E[3], double *const B[3],
                const double xi_in[3], double Ep[3], double Bp[3])
{
    double xi[3] = {xi_in[0], g->dim == 2 ? 0.0 : xi_in[1], xi_in[2]};
    for (int c = 0; c < 3; ++c) {
        double se[3], sb[3];
        for (int d = 0; d < 3; ++d) {
            se[d] = (d == c) ? 0.5 : 0.0;   /* E_c staggered along c */
            sb[d] = (d == c) ? 0.0 : 0.5;   /* B_c staggered across c */
        }
        if (g->dim == 2) { se[1] = 0.0; sb[1] = 0.0; }
        Ep[c] = gather_one(g, E[c], xi, se);
        Bp[c] = gather_one(g, B[c], xi, sb);
    }
}

/* ---------------------------------------------------------------- push */

/* Relativistic Boris scheme: half electric kick, magnetic rotation through
 * the t and s vectors, half electric kick (Boris 1970). */
void orc_boris(double q, double m, double dt, const double Ep[3],
               const double Bp[3], double u[3])
{
    const double h = q * dt / (2.0 * m);
    double um[3], t[3], s[3], up[3], uplus[3];
    for (int d = 0; d < 3; ++d) um[d] = u[d] + h * Ep[d];
    double gm = sqrt(1.0 + um[0] * um[0] + um[1] * um[1] + um[2] * um[2]);
    for (int d = 0; d < 3; ++d) t[d] = h * Bp[d] / gm;
    double t2 = t[0] * t[0] + t[1] * t[1] + t[2] * t[2];
    for (int d = 0; d < 3; ++d) s[d] = 2.0 * t[d] / (1.0 + t2);
    up[0] = um[0] + (um[1] * t[2] - um[2] * t[1]);
    up[1] = um[1] + (um[2] * t[0] - um[0] * t[2]);
    up[2] = um[2] + (um[0] * t[1] - um[1] * t[0]);
    uplus[0] = um[0] + (up[1] * s[2] - up[2] * s[1]);
    uplus[1] = um[1] + (up[2] * s[0] - up[0] * s[2]);
    uplus[2] = um[2] + (up[0] * s[1] - up[1] * s[0]);
    for (int d = 0; d < 3; ++d) u[d] = uplus[d] + h * Ep[d];
}

/* ---------------------------------------------------------------- deposit */

#define WMAX 8

/* Per-axis node window covering both positions: S0, dS = S1 - S0 on nodes
 * lo .. lo+len-1. */
static int axis_window(int32_t order, double x0, double x1, int64_t *lo,
                       double S0[WMAX], double dS[WMAX])
{
    double a = x0 < x1 ? x0 : x1, b = x0 < x1 ? x1 : x0;
    int64_t l = (int64_t)floor(a - 0.5 * (order + 1));
    int64_t h = (int64_t)floor(b + 0.5 * (order + 1));
    int len = (int)(h - l + 1);
    for (int t = 0; t < len; ++t) {
        double node = (double)(l + t);
        S0[t] = orc_shape(order, x0 - node);
        dS[t] = orc_shape(order, x1 - node) - S0[t];
    }
    *lo = l;
    return len;
}

/* Esirkepov's decomposition of the change of the particle's charge cloud
 * into three "flux" weights W^x, W^y, W^z, each integrated along its own
 * axis starting from zero left of the window.  The flux through the edge
 * right of the last window node is the sum of all dS along the line, zero
 * by the partition of unity, and is not written. */
void orc_deposit(const orc_grid *g, double *J[3], double q, double w,
                 const double x0[3], const double x1[3], double vy)
{
    const int32_t o = g->order;
    const double dx = g->dx[0], dy = g->dx[1], dz = g->dx[2], dt = g->dt;
    const double dV = dx * dy * dz;
    double S0x[WMAX], dSx[WMAX], S0y[WMAX], dSy[WMAX], S0z[WMAX], dSz[WMAX];
    int64_t lx, ly, lz;
    int nx = axis_window(o, x0[0], x1[0], &lx, S0x, dSx);
    int nz = axis_window(o, x0[2], x1[2], &lz, S0z, dSz);

    if (g->dim == 2) {
        const double cx = -q * w / (dt * dy * dz);
        const double cz = -q * w / (dt * dx * dy);
        const double cy = q * w * vy / dV;
        /* Jx: integrate W^x = dSx (S0z + dSz/2) along x. */
        for (int k = 0; k < nz; ++k) {
            double acc = 0.0;
            for (int i = 0; i < nx - 1; ++i) {
                acc += dSx[i] * (S0z[k] + 0.5 * dSz[k]);
                J[0][cell_index(g, lx + i, 0, lz + k)] += cx * acc;
            }
        }
        /* Jz: integrate W^z = dSz (S0x + dSx/2) along z. */
        for (int i = 0; i < nx; ++i) {
            double acc = 0.0;
            for (int k = 0; k < nz - 1; ++k) {
                acc += dSz[k] * (S0x[i] + 0.5 * dSx[i]);
                J[2][cell_index(g, lx + i, 0, lz + k)] += cz * acc;
            }
        }
        /* Jy (out of plane): charge moved with v_y, weighted by the
         * time-averaged in-plane shape product. */
        for (int k = 0; k < nz; ++k)
            for (int i = 0; i < nx; ++i) {
                double avg = S0x[i] * S0z[k] + 0.5 * dSx[i] * S0z[k] +
                             0.5 * S0x[i] * dSz[k] + dSx[i] * dSz[k] / 3.0;
                J[1][cell_index(g, lx + i, 0, lz + k)] += cy * avg;
            }
        return;
    }

    int ny = axis_window(o, x0[1], x1[1], &ly, S0y, dSy);
    const double cx = -q * w / (dt * dy * dz);
    const double cy = -q * w / (dt * dx * dz);
    const double cz = -q * w / (dt * dx * dy);
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j) {
            double acc = 0.0;
            for (int i = 0; i < nx - 1; ++i) {
                acc += dSx[i] * (S0y[j] * S0z[k] + 0.5 * dSy[j] * S0z[k] +
                                 0.5 * S0y[j] * dSz[k] + dSy[j] * dSz[k] / 3.0);
                J[0][cell_index(g, lx + i, ly + j, lz + k)] += cx * acc;
            }
        }
    for (int k = 0; k < nz; ++k)
        for (int i = 0; i < nx; ++i) {
            double acc = 0.0;
            for (int j = 0; j < ny - 1; ++j) {
                acc += dSy[j] * (S0z[k] * S0x[i] + 0.5 * dSz[k] * S0x[i] +
                                 0.5 * S0z[k] * dSx[i] + dSz[k] * dSx[i] / 3.0);
                J[1][cell_index(g, lx + i, ly + j, lz + k)] += cy * acc;
            }
        }
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            double acc = 0.0;
            for (int k = 0; k < nz - 1; ++k) {
                acc += dSz[k] * (S0x[i] * S0y[j] + 0.5 * dSx[i] * S0y[j] +
                                 0.5 * S0x[i] * dSy[j] + dSx[i] * dSy[j] / 3.0);
                J[2][cell_index(g, lx + i, ly + j, lz + k)] += cz * acc;
            }
        }
}

/* ---------------------------------------------------------------- Yee */

/* B -= h curl E, curl E taken at the B points.  In 2D the d/dy terms are
 * absent. */
void orc_faraday(const orc_grid *g, double *const E[3], double *B[3], double h)
{
    const int64_t n0 = g->n[0], n1 = g->n[1], n2 = g->n[2];
    const double dx = g->dx[0], dy = g->dx[1], dz = g->dx[2];
    const int has_y = (g->dim == 3);
    const int64_t N = n0 * n1 * n2;
    double *cx = calloc((size_t)N, sizeof(double));
    double *cy = calloc((size_t)N, sizeof(double));
    double *cz = calloc((size_t)N, sizeof(double));
    for (int64_t k = 0; k < n2; ++k)
        for (int64_t j = 0; j < n1; ++j)
            for (int64_t i = 0; i < n0; ++i) {
                int64_t c = cell_index(g, i, j, k);
                int64_t ip = cell_index(g, i + 1, j, k);
                int64_t jp = cell_index(g, i, j + 1, k);
                int64_t kp = cell_index(g, i, j, k + 1);
                double dEz_dy = has_y ? (E[2][jp] - E[2][c]) / dy : 0.0;
                double dEx_dy = has_y ? (E[0][jp] - E[0][c]) / dy : 0.0;
                cx[c] = dEz_dy - (E[1][kp] - E[1][c]) / dz;
                cy[c] = (E[0][kp] - E[0][c]) / dz - (E[2][ip] - E[2][c]) / dx;
                cz[c] = (E[1][ip] - E[1][c]) / dx - dEx_dy;
            }
    for (int64_t c = 0; c < N; ++c) {
        B[0][c] -= h * cx[c];
        B[1][c] -= h * cy[c];
        B[2][c] -= h * cz[c];
    }
    free(cx); free(cy); free(cz);
}

/* E += dt (curl B - J), curl B taken at the E points. */
void orc_ampere(const orc_grid *g, double *E[3], double *const B[3],
                double *const J[3], double dt)
{
    const int64_t n0 = g->n[0], n1 = g->n[1], n2 = g->n[2];
    const double dx = g->dx[0], dy = g->dx[1], dz = g->dx[2];
    const int has_y = (g->dim == 3);
    const int64_t N = n0 * n1 * n2;
    double *cx = calloc((size_t)N, sizeof(double));
    double *cy = calloc((size_t)N, sizeof(double));
    double *cz = calloc((size_t)N, sizeof(double));
    for (int64_t k = 0; k < n2; ++k)
        for (int64_t j = 0; j < n1; ++j)
            for (int64_t i = 0; i < n0; ++i) {
                int64_t c = cell_index(g, i, j, k);
                int64_t im = cell_index(g, i - 1, j, k);
                int64_t jm = cell_index(g, i, j - 1, k);
                int64_t km = cell_index(g, i, j, k - 1);
                double dBz_dy = has_y ? (B[2][c] - B[2][jm]) / dy : 0.0;
                double dBx_dy = has_y ? (B[0][c] - B[0][jm]) / dy : 0.0;
                cx[c] = dBz_dy - (B[1][c] - B[1][km]) / dz;
                cy[c] = (B[0][c] - B[0][km]) / dz - (B[2][c] - B[2][im]) / dx;
                cz[c] = (B[1][c] - B[1][im]) / dx - dBx_dy;
            }
    for (int64_t c = 0; c < N; ++c) {
        E[0][c] += dt * (cx[c] - J[0][c]);
        E[1][c] += dt * (cy[c] - J[1][c]);
        E[2][c] += dt * (cz[c] - J[2][c]);
    }
    free(cx); free(cy); free(cz);
}

void orc_fdtd_step(const orc_grid *g, double *E[3], double *B[3],
                   double *const J[3])
{
    orc_faraday(g, E, B, 0.5 * g->dt);
    orc_ampere(g, E, B, J, g->dt);
    orc_faraday(g, E, B, 0.5 * g->dt);
}

/* ---------------------------------------------------------------- step */

/* Wrap into [0, L); a sum that rounds to L itself is the point 0. */
double orc_wrap(double x, double L)
{
    if (x >= L) x -= L;
    if (x < 0.0) x += L;
    if (x >= L) x = 0.0;
    return x;
}

void orc_particles_step(const orc_grid *g, double *const E[3],
                        double *const B[3], double *J[3],
                        orc_species *sp, int32_t nsp)
{
    const int64_t N = (int64_t)g->n[0] * g->n[1] * g->n[2];
    for (int c = 0; c < 3; ++c) memset(J[c], 0, (size_t)N * sizeof(double));
    for (int32_t s = 0; s < nsp; ++s) {
        orc_species *S = &sp[s];
        for (int64_t p = 0; p < S->np; ++p) {
            double x0[3], x1[3], Ep[3], Bp[3], u[3];
            for (int d = 0; d < 3; ++d) {
                x0[d] = (g->dim == 2 && d == 1) ? 0.0 : S->x[d][p];
                u[d] = S->u[d][p];
            }
            orc_gather(g, E, B, x0, Ep, Bp);
            orc_boris(S->q, S->m, g->dt, Ep, Bp, u);
            double gam = sqrt(1.0 + u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
            for (int d = 0; d < 3; ++d)
                x1[d] = x0[d] + g->dt * u[d] / (gam * g->dx[d]);
            if (g->dim == 2) x1[1] = 0.0;
            orc_deposit(g, J, S->q, S->w[p], x0, x1, u[1] / gam);
            for (int d = 0; d < 3; ++d) {
                S->u[d][p] = u[d];
                if (g->dim == 2 && d == 1) continue;
                S->x[d][p] = orc_wrap(x1[d], (double)g->n[d]);
            }
        }
    }
}

void orc_pic_step(const orc_grid *g, double *E[3], double *B[3], double *J[3],
                  orc_species *sp, int32_t nsp)
{
    orc_particles_step(g, E, B, J, sp, nsp);
    orc_fdtd_step(g, E, B, J);
}

/* ---------------------------------------------------------------- checks */

void orc_rho(const orc_grid *g, double *rho, const orc_species *S)
{
    const int32_t o = g->order;
    const double dV = g->dx[0] * g->dx[1] * g->dx[2];
    for (int64_t p = 0; p < S->np; ++p) {
        double xi[3] = {S->x[0][p], g->dim == 2 ? 0.0 : S->x[1][p], S->x[2][p]};
        int64_t lo[3];
        for (int d = 0; d < 3; ++d) lo[d] = window_lo(o, xi[d], 0.0);
        int64_t jspan = (g->dim == 2) ? 0 : o + 2;
        for (int64_t k = lo[2]; k <= lo[2] + o + 2; ++k)
            for (int64_t j = lo[1]; j <= lo[1] + jspan; ++j)
                for (int64_t i = lo[0]; i <= lo[0] + o + 2; ++i) {
                    double sy = (g->dim == 2) ? 1.0 : orc_shape(o, xi[1] - (double)j);
                    double s = orc_shape(o, xi[0] - (double)i) * sy *
                               orc_shape(o, xi[2] - (double)k);
                    int64_t c = (g->dim == 2) ? cell_index(g, i, 0, k)
                                              : cell_index(g, i, j, k);
                    rho[c] += S->q * S->w[p] * s / dV;
                }
    }
}

void orc_div_j(const orc_grid *g, double *const J[3], double *divj)
{
    const int has_y = (g->dim == 3);
    for (int64_t k = 0; k < g->n[2]; ++k)
        for (int64_t j = 0; j < g->n[1]; ++j)
            for (int64_t i = 0; i < g->n[0]; ++i) {
                int64_t c = cell_index(g, i, j, k);
                double d = (J[0][c] - J[0][cell_index(g, i - 1, j, k)]) / g->dx[0] +
                           (J[2][c] - J[2][cell_index(g, i, j, k - 1)]) / g->dx[2];
                if (has_y)
                    d += (J[1][c] - J[1][cell_index(g, i, j - 1, k)]) / g->dx[1];
                divj[c] = d;
            }
}

/* Electromagnetic field energy 1/2 sum over cells of (E.E + B.B) dV in
 * these units (eps0 = mu0 = 1), every component sampled at its own Yee
 * point of the cell. */
double orc_field_energy(const orc_grid *g, double *const E[3],
                        double *const B[3])
{
    const int64_t N = (int64_t)g->n[0] * g->n[1] * g->n[2];
    const double dV = g->dx[0] * g->dx[1] * g->dx[2];
    double s = 0.0;
    for (int c = 0; c < 3; ++c)
        for (int64_t i = 0; i < N; ++i)
            s += E[c][i] * E[c][i] + B[c][i] * B[c][i];
    return 0.5 * s * dV;
}

/* Relativistic kinetic energy m (gamma - 1) c^2 per physical particle,
 * times the weight.  gamma - 1 is evaluated as u.u / (1 + gamma), the same
 * quantity without the cancellation of sqrt(1 + u.u) - 1 at |u| << 1. */
double orc_kinetic_energy(const orc_species *S)
{
    double s = 0.0;
    for (int64_t p = 0; p < S->np; ++p) {
        double u2 = S->u[0][p] * S->u[0][p] + S->u[1][p] * S->u[1][p] +
                    S->u[2][p] * S->u[2][p];
        s += S->w[p] * S->m * (u2 / (1.0 + sqrt(1.0 + u2)));
    }
    return s;
}

/* ---------------------------------------------------------------- sort */

void orc_tile_keys(const orc_grid *g, const int32_t tile[3],
                   const orc_species *S, int32_t *key)
{
    int64_t nt[3];
    for (int d = 0; d < 3; ++d) nt[d] = (g->n[d] + tile[d] - 1) / tile[d];
    for (int64_t p = 0; p < S->np; ++p) {
        int64_t t[3];
        for (int d = 0; d < 3; ++d) {
            if (g->dim == 2 && d == 1) { t[d] = 0; continue; }
            int64_t c = (int64_t)floor(S->x[d][p]);
            c = wrapi(c, g->n[d]);
            t[d] = c / tile[d];
        }
        key[p] = (int32_t)(t[0] + nt[0] * (t[1] + nt[1] * t[2]));
    }
}

static const int32_t *g_sort_key;

static int by_key_then_index(const void *a, const void *b)
{
    int32_t ia = *(const int32_t *)a, ib = *(const int32_t *)b;
    int32_t ka = g_sort_key[ia], kb = g_sort_key[ib];
    if (ka != kb) return ka < kb ? -1 : 1;
    return ia < ib ? -1 : (ia > ib ? 1 : 0);
}

void orc_cell_order_keys(const orc_grid *g, const int32_t tile[3], int32_t cbits,
                         const orc_species *S, int64_t *key)
{
    int64_t nt[3];
    for (int d = 0; d < 3; ++d) nt[d] = (g->n[d] + tile[d] - 1) / tile[d];
    const int64_t t1 = g->dim == 3 ? tile[1] : 1;
    for (int64_t p = 0; p < S->np; ++p) {
        int64_t t[3], l[3];
        for (int d = 0; d < 3; ++d) {
            if (g->dim == 2 && d == 1) { t[d] = 0; l[d] = 0; continue; }
            int64_t c = wrapi((int64_t)floor(S->x[d][p]), g->n[d]);
            t[d] = c / tile[d];
            l[d] = c - t[d] * tile[d];
        }
        const int64_t id = t[0] + nt[0] * (t[1] + nt[1] * t[2]);
        const int64_t cls = (l[0] + l[1] + l[2]) % 4;
        const int64_t within = l[0] + tile[0] * (l[1] + t1 * l[2]);
        key[p] = (id << (cbits + 2)) | (cls << cbits) | within;
    }
}

void orc_tile_cell_keys(const orc_grid *g, const int32_t tile[3], int32_t cbits,
                        const orc_species *S, int64_t *key)
{
    int64_t nt[3];
    for (int d = 0; d < 3; ++d) nt[d] = (g->n[d] + tile[d] - 1) / tile[d];
    const int64_t t1 = g->dim == 3 ? tile[1] : 1;
    for (int64_t p = 0; p < S->np; ++p) {
        int64_t t[3], l[3];
        for (int d = 0; d < 3; ++d) {
            if (g->dim == 2 && d == 1) { t[d] = 0; l[d] = 0; continue; }
            int64_t c = wrapi((int64_t)floor(S->x[d][p]), g->n[d]);
            t[d] = c / tile[d];
            l[d] = c - t[d] * tile[d];
        }
        const int64_t id = t[0] + nt[0] * (t[1] + nt[1] * t[2]);
        key[p] = (id << cbits) | (l[0] + tile[0] * (l[1] + t1 * l[2]));
    }
}

static const int64_t *g_sort_key64;

static int by_key64_then_index(const void *a, const void *b)
{
    int32_t ia = *(const int32_t *)a, ib = *(const int32_t *)b;
    int64_t ka = g_sort_key64[ia], kb = g_sort_key64[ib];
    if (ka != kb) return ka < kb ? -1 : 1;
    return ia < ib ? -1 : (ia > ib ? 1 : 0);
}

void orc_stable_perm(int64_t np, const int64_t *key, int32_t *perm)
{
    for (int64_t p = 0; p < np; ++p) perm[p] = (int32_t)p;
    g_sort_key64 = key;
    qsort(perm, (size_t)np, sizeof(int32_t), by_key64_then_index);
}

void orc_quad_order(int64_t np, const int64_t *key, int32_t cbits, int32_t *perm)
{
    int32_t *sorted = (int32_t *)malloc(sizeof(int32_t) * (size_t)(np > 0 ? np : 1));
    char *rest = (char *)malloc((size_t)(np > 0 ? np : 1));
    orc_stable_perm(np, key, sorted);
    /* runs of equal keys: mark each cell's last count mod 4 */
    for (int64_t a = 0; a < np;) {
        int64_t b = a;
        while (b < np && key[sorted[b]] == key[sorted[a]]) ++b;
        const int64_t cnt = b - a;
        for (int64_t i = a; i < b; ++i) rest[i] = (i - a) >= cnt - cnt % 4;
        a = b;
    }
    /* per tile: whole groups first, then the rest */
    int64_t out = 0;
    for (int64_t a = 0; a < np;) {
        const int64_t tile = key[sorted[a]] >> (cbits + 2);
        int64_t b = a;
        while (b < np && (key[sorted[b]] >> (cbits + 2)) == tile) ++b;
        for (int64_t i = a; i < b; ++i) if (!rest[i]) perm[out++] = sorted[i];
        for (int64_t i = a; i < b; ++i) if (rest[i]) perm[out++] = sorted[i];
        a = b;
    }
    free(rest);
    free(sorted);
}

/* Rank-major order inside each tile (tile id = key >> cbits, key as
 * orc_tile_cell_keys): sorted by key (ties in index order), each particle's
 * rank is its place among the particles of its cell (0, 1, ...; ranks
 * above 2^rbits - 1 count as 2^rbits - 1); then every tile is ordered by
 * rank, ties kept in cell order.  Consecutive particles of one rank sit in
 * consecutive cells.  A layout choice of the GPU sort. */
void orc_rank_major(int64_t np, const int64_t *key, int32_t cbits, int32_t rbits, int32_t *perm)
{
    int32_t *sorted = (int32_t *)malloc(sizeof(int32_t) * (size_t)(np > 0 ? np : 1));
    int64_t *key2 = (int64_t *)malloc(sizeof(int64_t) * (size_t)(np > 0 ? np : 1));
    int32_t *order = (int32_t *)malloc(sizeof(int32_t) * (size_t)(np > 0 ? np : 1));
    orc_stable_perm(np, key, sorted);
    const int64_t rmax = ((int64_t)1 << rbits) - 1;
    for (int64_t a = 0; a < np;) {
        int64_t b = a;
        while (b < np && key[sorted[b]] == key[sorted[a]]) ++b;
        for (int64_t i = a; i < b; ++i) {
            const int64_t rank = (i - a) < rmax ? (i - a) : rmax;
            key2[i] = ((key[sorted[i]] >> cbits) << rbits) | rank;
        }
        a = b;
    }
    /* stable sort of the sorted positions by key2 */
    orc_stable_perm(np, key2, order);
    for (int64_t i = 0; i < np; ++i) perm[i] = sorted[order[i]];
    free(order);
    free(key2);
    free(sorted);
}

void orc_stable_sort(int64_t np, const int32_t *key, int32_t nkeys,
                     int32_t *perm, int32_t *count, int32_t *offset)
{
    for (int64_t p = 0; p < np; ++p) perm[p] = (int32_t)p;
    g_sort_key = key;
    qsort(perm, (size_t)np, sizeof(int32_t), by_key_then_index);
    for (int32_t t = 0; t < nkeys; ++t) count[t] = 0;
    for (int64_t p = 0; p < np; ++p) count[key[p]]++;
    offset[0] = 0;
    for (int32_t t = 0; t < nkeys; ++t) offset[t + 1] = offset[t] + count[t];
}

/* ---------------------------------------------------------------- boundaries
 *
 * Absorbing layers at the two ends of the z axis (the laser's axis): the
 * Maxwell equations with an electric and an equal magnetic conductivity,
 *   dE/dt + sigma E = curl B - J,   dB/dt + sigma B = -curl E,
 * whose impedance equals that of vacuum (eps0 = mu0 = 1), so a wave at
 * normal incidence enters without reflection in the continuum limit and
 * decays as exp(-integral sigma dz).  sigma(z) = sigma_max (d / L)^p at
 * depth d into a layer of L cells (0 outside the layers), each field
 * component taking sigma at its own Yee point along z.  In time each
 * sub-step integrates the decay exactly: over a step tau,
 *   F <- exp(-sigma tau) F + (1 - exp(-sigma tau)) / sigma * S,
 * S the curl source of that sub-step (tau S when sigma = 0: plain Yee). */

double orc_absorber_sigma(const orc_absorber *a, double z, double nz)
{
    const double L = (double)a->cells;
    if (a->cells <= 0) return 0.0;
    double d = 0.0;
    if (z < L) d = L - z;
    else if (z > nz - L) d = z - (nz - L);
    if (d <= 0.0) return 0.0;
    return a->sigma_max * pow(d / L, (double)a->power);
}

/* decay factor and source weight of one sub-step of length tau */
static void absorb_coef(double sigma, double tau, double *alpha, double *beta)
{
    if (sigma == 0.0) {
        *alpha = 1.0;
        *beta = tau;
    } else {
        *alpha = exp(-sigma * tau);
        *beta = (1.0 - *alpha) / sigma;
    }
}

/* z of a component's Yee point in cell k: E_x, E_y, B_z at k; E_z, B_x, B_y
 * at k + 1/2 (comp 0..2 = E, 3..5 = B). */
static double comp_z(int comp, int64_t k)
{
    const int half = (comp == 2 || comp == 3 || comp == 4);
    return (double)k + (half ? 0.5 : 0.0);
}

/* curl E at the B points (3 arrays of N), periodic; 2D: no d/dy terms */
static void curl_e(const orc_grid *g, double *const E[3], double *c[3])
{
    const int64_t n0 = g->n[0], n1 = g->n[1], n2 = g->n[2];
    const double dx = g->dx[0], dy = g->dx[1], dz = g->dx[2];
    const int has_y = (g->dim == 3);
    for (int64_t k = 0; k < n2; ++k)
        for (int64_t j = 0; j < n1; ++j)
            for (int64_t i = 0; i < n0; ++i) {
                int64_t q = cell_index(g, i, j, k);
                int64_t ip = cell_index(g, i + 1, j, k);
                int64_t jp = cell_index(g, i, j + 1, k);
                int64_t kp = cell_index(g, i, j, k + 1);
                double dEz_dy = has_y ? (E[2][jp] - E[2][q]) / dy : 0.0;
                double dEx_dy = has_y ? (E[0][jp] - E[0][q]) / dy : 0.0;
                c[0][q] = dEz_dy - (E[1][kp] - E[1][q]) / dz;
                c[1][q] = (E[0][kp] - E[0][q]) / dz - (E[2][ip] - E[2][q]) / dx;
                c[2][q] = (E[1][ip] - E[1][q]) / dx - dEx_dy;
            }
}

/* curl B at the E points */
static void curl_b(const orc_grid *g, double *const B[3], double *c[3])
{
    const int64_t n0 = g->n[0], n1 = g->n[1], n2 = g->n[2];
    const double dx = g->dx[0], dy = g->dx[1], dz = g->dx[2];
    const int has_y = (g->dim == 3);
    for (int64_t k = 0; k < n2; ++k)
        for (int64_t j = 0; j < n1; ++j)
            for (int64_t i = 0; i < n0; ++i) {
                int64_t q = cell_index(g, i, j, k);
                int64_t im = cell_index(g, i - 1, j, k);
                int64_t jm = cell_index(g, i, j - 1, k);
                int64_t km = cell_index(g, i, j, k - 1);
                double dBz_dy = has_y ? (B[2][q] - B[2][jm]) / dy : 0.0;
                double dBx_dy = has_y ? (B[0][q] - B[0][jm]) / dy : 0.0;
                c[0][q] = dBz_dy - (B[1][q] - B[1][km]) / dz;
                c[1][q] = (B[0][q] - B[0][km]) / dz - (B[2][q] - B[2][im]) / dx;
                c[2][q] = (B[1][q] - B[1][im]) / dx - dBx_dy;
            }
}

static void faraday_abs(const orc_grid *g, double *const E[3], double *B[3], double h,
                        const orc_absorber *a, double zoff)
{
    const int64_t n0 = g->n[0], n1 = g->n[1], n2 = g->n[2];
    const int64_t N = n0 * n1 * n2;
    double *cu[3];
    for (int c = 0; c < 3; ++c) cu[c] = malloc((size_t)N * sizeof(double));
    curl_e(g, E, cu);
    for (int64_t k = 0; k < n2; ++k)
        for (int c = 0; c < 3; ++c) {
            const double z = fmod(comp_z(3 + c, k) - zoff + 2.0 * (double)n2, (double)n2);
            double al, be;
            absorb_coef(orc_absorber_sigma(a, z, (double)n2), h, &al, &be);
            for (int64_t r = 0; r < n0 * n1; ++r) {
                const int64_t i = k * n0 * n1 + r;
                B[c][i] = al * B[c][i] - be * cu[c][i];
            }
        }
    for (int c = 0; c < 3; ++c) free(cu[c]);
}

static void ampere_abs(const orc_grid *g, double *E[3], double *const B[3], double *const J[3],
                       double dt, const orc_absorber *a, double zoff)
{
    const int64_t n0 = g->n[0], n1 = g->n[1], n2 = g->n[2];
    const int64_t N = n0 * n1 * n2;
    double *cu[3];
    for (int c = 0; c < 3; ++c) cu[c] = malloc((size_t)N * sizeof(double));
    curl_b(g, B, cu);
    for (int64_t k = 0; k < n2; ++k)
        for (int c = 0; c < 3; ++c) {
            const double z = fmod(comp_z(c, k) - zoff + 2.0 * (double)n2, (double)n2);
            double al, be;
            absorb_coef(orc_absorber_sigma(a, z, (double)n2), dt, &al, &be);
            for (int64_t r = 0; r < n0 * n1; ++r) {
                const int64_t i = k * n0 * n1 + r;
                E[c][i] = al * E[c][i] + be * (cu[c][i] - J[c][i]);
            }
        }
    for (int c = 0; c < 3; ++c) free(cu[c]);
}

void orc_fdtd_step_absorb(const orc_grid *g, double *E[3], double *B[3], double *const J[3],
                          const orc_absorber *a, double zoff)
{
    faraday_abs(g, E, B, 0.5 * g->dt, a, zoff);
    ampere_abs(g, E, B, J, g->dt, a, zoff);
    faraday_abs(g, E, B, 0.5 * g->dt, a, zoff);
}

/* Laser antenna: a sheet of current in the plane of the E_x points at
 * z = k_a (cell k_a), K_x(x, y, t) = -2 E0 exp(-r^2 / w^2) g(t) sin(w0 (t -
 * t0)), g(t) = exp(-((t - t0) / tau)^2), r measured from (x0, y0) at each
 * E_x point (i + 1/2, j).  A current sheet K radiates E = -K / 2 to both
 * sides (c = eps0 = 1), so the emitted field has amplitude E0.  Added as a
 * volume current K / dz in cell layer k_a, at time t (the caller passes the
 * half-step time of the J it is added to). */
void orc_antenna_add(const orc_grid *g, double *J[3], const orc_antenna *an, double t)
{
    const int64_t n0 = g->n[0], n1 = g->n[1];
    const double s = (t - an->t0) / an->tau;
    const double amp = -2.0 * an->E0 * exp(-s * s) * sin(an->omega * (t - an->t0)) / g->dx[2];
    for (int64_t j = 0; j < n1; ++j)
        for (int64_t i = 0; i < n0; ++i) {
            const double x = ((double)i + 0.5) * g->dx[0] - an->x0;
            const double y = (g->dim == 3) ? (double)j * g->dx[1] - an->y0 : 0.0;
            const double r2 = x * x + y * y;
            J[0][cell_index(g, i, j, an->k)] += amp * exp(-r2 / (an->waist * an->waist));
        }
}

/* Moving window, one cell along +z: every field array moves one cell toward
 * -z (F(k) <- F(k + 1)), the new top layer starts at zero; particles move
 * one cell toward -z in the window frame and those that leave it (z < 0)
 * are removed, the others keeping their order.  Returns the new count of
 * the species (its arrays compacted in place). */
int64_t orc_window_shift_particles(const orc_grid *g, orc_species *sp)
{
    int64_t m = 0;
    for (int64_t p = 0; p < sp->np; ++p) {
        const double z = sp->x[2][p] - 1.0;
        if (z < 0.0) continue;
        for (int d = 0; d < 3; ++d) {
            if (d != 1 || g->dim == 3) sp->x[d][m] = sp->x[d][p];
            sp->u[d][m] = sp->u[d][p];
        }
        sp->x[2][m] = z;
        sp->w[m] = sp->w[p];
        ++m;
    }
    sp->np = m;
    return m;
}

void orc_window_shift_fields(const orc_grid *g, double *E[3], double *B[3])
{
    const int64_t plane = (int64_t)g->n[0] * g->n[1];
    const int64_t N = plane * g->n[2];
    for (int c = 0; c < 3; ++c) {
        memmove(E[c], E[c] + plane, (size_t)(N - plane) * sizeof(double));
        memmove(B[c], B[c] + plane, (size_t)(N - plane) * sizeof(double));
        memset(E[c] + N - plane, 0, (size_t)plane * sizeof(double));
        memset(B[c] + N - plane, 0, (size_t)plane * sizeof(double));
    }
}

/* ---------------------------------------------------------------- electrostatic
 *
 * The electrostatic variant of the step: the field is E = -grad phi with
 * the discrete Poisson equation div grad phi = -(rho - <rho>) (the mean
 * removed: a neutralising background) solved elsewhere; B = 0.  Each
 * particle gathers E at x^n (shapes and stagger as orc_gather), takes the
 * Boris step (with B = 0 a pure kick u += q E dt / m), advances and wraps;
 * no current is deposited. */

/* E = -grad phi at the Yee E points: E_x(i+1/2, j, k) = -(phi(i+1) -
 * phi(i)) / dx, and likewise along y and z (2D: E_y = 0). */
void orc_es_field(const orc_grid *g, const double *phi, double *E[3])
{
    const int has_y = (g->dim == 3);
    for (int64_t k = 0; k < g->n[2]; ++k)
        for (int64_t j = 0; j < g->n[1]; ++j)
            for (int64_t i = 0; i < g->n[0]; ++i) {
                const int64_t c = cell_index(g, i, j, k);
                E[0][c] = -(phi[cell_index(g, i + 1, j, k)] - phi[c]) / g->dx[0];
                E[1][c] = has_y ? -(phi[cell_index(g, i, j + 1, k)] - phi[c]) / g->dx[1] : 0.0;
                E[2][c] = -(phi[cell_index(g, i, j, k + 1)] - phi[c]) / g->dx[2];
            }
}

void orc_es_particles_step(const orc_grid *g, double *const E[3], orc_species *sp, int32_t nsp)
{
    const int64_t N = (int64_t)g->n[0] * g->n[1] * g->n[2];
    double *zero = calloc((size_t)N, sizeof(double));
    double *Bz[3] = {zero, zero, zero};
    for (int32_t s = 0; s < nsp; ++s) {
        orc_species *S = &sp[s];
        for (int64_t p = 0; p < S->np; ++p) {
            double x0[3], Ep[3], Bp[3], u[3];
            for (int d = 0; d < 3; ++d) {
                x0[d] = (g->dim == 2 && d == 1) ? 0.0 : S->x[d][p];
                u[d] = S->u[d][p];
            }
            orc_gather(g, E, Bz, x0, Ep, Bp);
            orc_boris(S->q, S->m, g->dt, Ep, Bp, u);
            const double gam = sqrt(1.0 + u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
            for (int d = 0; d < 3; ++d) {
                S->u[d][p] = u[d];
                if (g->dim == 2 && d == 1) continue;
                S->x[d][p] = orc_wrap(x0[d] + g->dt * u[d] / (gam * g->dx[d]), (double)g->n[d]);
            }
        }
    }
    free(zero);
}

/* ---------------------------------------------------------------- variants
 *
 * Two published variants of the particle update, selectable beside the
 * defaults: the relativistic pusher of Vay (Phys. Plasmas 15, 056701,
 * 2008), whose u^(n+1/2) makes E + v x B vanish exactly for a particle at
 * the E x B drift velocity (Boris's average does not at relativistic
 * speeds), and the "Galerkin" gather, which lowers the shape order by one
 * along every axis on which a field component sits at half-integer points
 * (the order-0 shape being the nearest node). */

void orc_vay(double q, double m, double dt, const double Ep[3], const double Bp[3], double u[3])
{
    const double qdt = q * dt / m;
    const double g0 = sqrt(1.0 + u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
    const double v0[3] = {u[0] / g0, u[1] / g0, u[2] / g0};
    /* u' = u + (q dt / m) (E + v x B / 2) */
    double up[3];
    up[0] = u[0] + qdt * (Ep[0] + 0.5 * (v0[1] * Bp[2] - v0[2] * Bp[1]));
    up[1] = u[1] + qdt * (Ep[1] + 0.5 * (v0[2] * Bp[0] - v0[0] * Bp[2]));
    up[2] = u[2] + qdt * (Ep[2] + 0.5 * (v0[0] * Bp[1] - v0[1] * Bp[0]));
    const double tau[3] = {0.5 * qdt * Bp[0], 0.5 * qdt * Bp[1], 0.5 * qdt * Bp[2]};
    const double tau2 = tau[0] * tau[0] + tau[1] * tau[1] + tau[2] * tau[2];
    const double ustar = up[0] * tau[0] + up[1] * tau[1] + up[2] * tau[2];
    const double gp2 = 1.0 + up[0] * up[0] + up[1] * up[1] + up[2] * up[2];
    const double sigma = gp2 - tau2;
    const double g1 = sqrt(0.5 * (sigma + sqrt(sigma * sigma + 4.0 * (tau2 + ustar * ustar))));
    const double t[3] = {tau[0] / g1, tau[1] / g1, tau[2] / g1};
    const double s = 1.0 / (1.0 + t[0] * t[0] + t[1] * t[1] + t[2] * t[2]);
    const double ut = up[0] * t[0] + up[1] * t[1] + up[2] * t[2];
    u[0] = s * (up[0] + ut * t[0] + (up[1] * t[2] - up[2] * t[1]));
    u[1] = s * (up[1] + ut * t[1] + (up[2] * t[0] - up[0] * t[2]));
    u[2] = s * (up[2] + ut * t[2] + (up[0] * t[1] - up[1] * t[0]));
}

/* shape of order `order` along one axis; order 0: the nearest node,
 * 1 for -1/2 <= a < 1/2 */
static double shape_any(int32_t order, double a)
{
    if (order == 0) return (a >= -0.5 && a < 0.5) ? 1.0 : 0.0;
    return orc_shape(order, a);
}

static double gather_galerkin_one(const orc_grid *g, const double *F, const double xi[3],
                                  const double st[3])
{
    int32_t o[3];
    int64_t lo[3];
    for (int d = 0; d < 3; ++d) {
        o[d] = st[d] != 0.0 ? g->order - 1 : g->order;
        lo[d] = (int64_t)floor(xi[d] - st[d] - 0.5 * (o[d] + 1)) - 1;
    }
    double sum = 0.0;
    const int64_t jlo = g->dim == 2 ? 0 : lo[1], jhi = g->dim == 2 ? 0 : lo[1] + o[1] + 3;
    for (int64_t k = lo[2]; k <= lo[2] + o[2] + 3; ++k) {
        const double sz = shape_any(o[2], xi[2] - ((double)k + st[2]));
        for (int64_t j = jlo; j <= jhi; ++j) {
            const double sy = g->dim == 2 ? 1.0 : shape_any(o[1], xi[1] - ((double)j + st[1]));
            for (int64_t i = lo[0]; i <= lo[0] + o[0] + 3; ++i) {
                const double sx = shape_any(o[0], xi[0] - ((double)i + st[0]));
                sum += F[cell_index(g, i, j, k)] * sx * sy * sz;
            }
        }
    }
    return sum;
}

void orc_gather_galerkin(const orc_grid *g, double *const E[3], double *const B[3],
                         const double xi_in[3], double Ep[3], double Bp[3])
{
    double xi[3] = {xi_in[0], g->dim == 2 ? 0.0 : xi_in[1], xi_in[2]};
    for (int c = 0; c < 3; ++c) {
        double se[3], sb[3];
        for (int d = 0; d < 3; ++d) {
            se[d] = (d == c) ? 0.5 : 0.0;
            sb[d] = (d == c) ? 0.0 : 0.5;
        }
        if (g->dim == 2) { se[1] = 0.0; sb[1] = 0.0; }
        Ep[c] = gather_galerkin_one(g, E[c], xi, se);
        Bp[c] = gather_galerkin_one(g, B[c], xi, sb);
    }
}

/* orc_particles_step with the pusher (0 Boris, 1 Vay) and gather (0 the
 * same order on every stagger, 1 Galerkin) chosen. */
void orc_particles_step_opts(const orc_grid *g, double *const E[3], double *const B[3],
                             double *J[3], orc_species *sp, int32_t nsp, int32_t pusher,
                             int32_t gather)
{
    const int64_t N = (int64_t)g->n[0] * g->n[1] * g->n[2];
    for (int c = 0; c < 3; ++c) memset(J[c], 0, (size_t)N * sizeof(double));
    for (int32_t s = 0; s < nsp; ++s) {
        orc_species *S = &sp[s];
        for (int64_t p = 0; p < S->np; ++p) {
            double x0[3], x1[3], Ep[3], Bp[3], u[3];
            for (int d = 0; d < 3; ++d) {
                x0[d] = (g->dim == 2 && d == 1) ? 0.0 : S->x[d][p];
                u[d] = S->u[d][p];
            }
            if (gather) orc_gather_galerkin(g, E, B, x0, Ep, Bp);
            else orc_gather(g, E, B, x0, Ep, Bp);
            if (pusher) orc_vay(S->q, S->m, g->dt, Ep, Bp, u);
            else orc_boris(S->q, S->m, g->dt, Ep, Bp, u);
            double gam = sqrt(1.0 + u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
            for (int d = 0; d < 3; ++d)
                x1[d] = x0[d] + g->dt * u[d] / (gam * g->dx[d]);
            if (g->dim == 2) x1[1] = 0.0;
            orc_deposit(g, J, S->q, S->w[p], x0, x1, u[1] / gam);
            for (int d = 0; d < 3; ++d) {
                S->u[d][p] = u[d];
                if (g->dim == 2 && d == 1) continue;
                S->x[d][p] = orc_wrap(x1[d], (double)g->n[d]);
            }
        }
    }
}

/* ---------------------------------------------------------------- in-situ
 *
 * Moments of one species per cell layer along z of the window frame (layer
 * (k - zoff) mod n_z of array layer k): out[5 k + q], q = 0 sum w, 1..3
 * sum w u_d, 4 sum w m (gamma - 1) (gamma - 1 = u.u / (1 + gamma)); the
 * layer of a particle is floor(z) of its position.  Added into out. */
void orc_slice_moments(const orc_grid *g, const orc_species *S, int32_t zoff, double *out)
{
    const int64_t nz = g->n[2];
    for (int64_t p = 0; p < S->np; ++p) {
        int64_t k = (int64_t)floor(S->x[2][p]);
        k = ((k - zoff) % nz + nz) % nz;
        const double u0 = S->u[0][p], u1 = S->u[1][p], u2 = S->u[2][p];
        const double uu = u0 * u0 + u1 * u1 + u2 * u2;
        const double w = S->w[p];
        out[5 * k + 0] += w;
        out[5 * k + 1] += w * u0;
        out[5 * k + 2] += w * u1;
        out[5 * k + 3] += w * u2;
        out[5 * k + 4] += w * S->m * (uu / (1.0 + sqrt(1.0 + uu)));
    }
}
