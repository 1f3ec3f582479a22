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
