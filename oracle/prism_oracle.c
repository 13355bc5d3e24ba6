/*
 * prism_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow CPU evaluation of the sensitivity matrix G of Hogue, Renaut &
 * Vatankhah (arXiv 1912.06976), used only to check the GPU library.  Only the
 * test suite, the smoke check and the benchmark's CPU-baseline leg may load
 * it.  It shares no code, header or table with the GPU library.
 *
 * What it computes (Sec. 2, eq. continuousforwardmodel, eq. htilde; Table 3
 * of the appendix for coordinates):
 *   station (i, j), 0-based, at ((i + 1/2) dx, (j + 1/2) dy, -h), h >= 0;
 *   prism (p, q, r) spans [(p - pxl) dx, (p - pxl + 1) dx] x
 *                          [(q - pyl) dy, (q - pyl + 1) dy] x [z_r, z_{r+1}],
 *   z pointing down;  chi = x_edge - a_i, ups = y_edge - b_j, zeta = z_edge + h;
 *   G[k][l] = scale * sum_{corners} (-1)^(i+j+k) f(chi_i, ups_j, zeta_k),
 *   k = j sx + i,  l = r nx ny + q nx + p   (x fastest, eq. htilde).
 * Every entry is computed from the station and prism coordinates; nothing
 * here uses the Toeplitz structure, a circulant or an FFT.
 *
 * kind: 0 = gravity g_z (Sec. 4.1), 1 = magnetic total-field anomaly for
 * induced magnetisation (Sec. 4.2), 2 = an index probe whose entry is
 * (p - pxl - i) + 4096 (q - pyl - j) + 2^24 r, computed from the geometry,
 * 3 = sum_ab w_ab U_ab, a weighted sum of the second derivatives of the
 * prism's potential with respect to the station, each component from its own
 * closed form (a user-chosen kernel, Sec. 1 (vi)).
 *
 * Build: gcc -O2 -fopenmp -ffp-contract=off -shared -fPIC ... -lquadmath -lm
 * (no fast-math: IEEE round-to-nearest throughout).
 */
#include <math.h>
#include <quadmath.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ---- double instantiation of the corner terms ---- */
#define REAL double
#define SFX _d
#define R_SQRT sqrt
#define R_LOG log
#define R_ATAN atan
#define R_FABS fabs
#define R_SIN sin
#define R_COS cos
#define R_PI 3.14159265358979323846264338327950288
#include "prism_terms.inc"
#undef REAL
#undef SFX
#undef R_SQRT
#undef R_LOG
#undef R_ATAN
#undef R_FABS
#undef R_SIN
#undef R_COS
#undef R_PI

/* ---- __float128 instantiation ---- */
#define REAL __float128
#define SFX _q
#define R_SQRT sqrtq
#define R_LOG logq
#define R_ATAN atanq
#define R_FABS fabsq
#define R_SIN sinq
#define R_COS cosq
#define R_PI M_PIq
#include "prism_terms.inc"

typedef struct {
    int32_t kind;                 /* 0 gravity, 1 magnetic, 2 probe          */
    int32_t sx, sy, nz;           /* stations and depth layers               */
    int32_t pxl, pxr, pyl, pyr;   /* padding prisms on each side             */
    double dx, dy;                /* prism sizes [m]                         */
    double h;                     /* station height above z = 0 [m]          */
    const double *zedge;          /* nz + 1 increasing depths [m]            */
    double incl, decl;            /* magnetic field direction [deg]          */
    double scale;                 /* gamma (gravity) or F / (4 pi) (magnetic) */
    double w[6];                  /* kind 3: w_xx, w_yy, w_zz, w_xy, w_xz, w_yz */
} orc_problem;

/* the weights orc_prism takes for a problem: magnetic G_1..G_5 (kind 1), the
 * component weights (kind 3), zeros otherwise */
static void orc_weights_d(const orc_problem *P, double g[6])
{
    for (int t = 0; t < 6; ++t) g[t] = 0;
    if (P->kind == 1) orc_mag_weights_d(P->incl, P->decl, g);
    if (P->kind == 3) for (int t = 0; t < 6; ++t) g[t] = P->w[t];
}
static void orc_weights_q(const orc_problem *P, __float128 g[6])
{
    for (int t = 0; t < 6; ++t) g[t] = 0;
    if (P->kind == 1) orc_mag_weights_q(P->incl, P->decl, g);
    if (P->kind == 3) for (int t = 0; t < 6; ++t) g[t] = P->w[t];
}

static int orc_nx(const orc_problem *P) { return P->sx + P->pxl + P->pxr; }
static int orc_ny(const orc_problem *P) { return P->sy + P->pyl + P->pyr; }

/* Corner coordinates of prism (p,q,r) seen from station (i,j), from the
 * absolute coordinates of both (Table 3; Sec. 2.1.1-2.1.2). */
static void orc_corners(const orc_problem *P, int i, int j, int p, int q, int r, double b[6])
{
    double a = (i + 0.5) * P->dx, bb = (j + 0.5) * P->dy, c = -P->h;
    double x0 = (p - P->pxl) * P->dx, y0 = (q - P->pyl) * P->dy;
    b[0] = x0 - a;
    b[1] = (x0 + P->dx) - a;
    b[2] = y0 - bb;
    b[3] = (y0 + P->dy) - bb;
    b[4] = P->zedge[r] - c;
    b[5] = P->zedge[r + 1] - c;
}

static double orc_probe_value(const orc_problem *P, const double b[6], int r)
{
    /* offsets recovered from the geometry: chi1 = (p - pxl - i - 1/2) dx */
    double ox = nearbyint(b[0] / P->dx + 0.5);
    double oy = nearbyint(b[2] / P->dy + 0.5);
    return ox + 4096.0 * oy + 16777216.0 * r;
}

static double orc_entry_d(const orc_problem *P, const double g[6], int i, int j, int p, int q, int r,
                          double *abs_sum)
{
    double b[6];
    orc_corners(P, i, j, p, q, r, b);
    if (P->kind == 2) { if (abs_sum) *abs_sum = 0; return orc_probe_value(P, b, r); }
    double a = 0;
    double v = orc_prism_d(P->kind, b, g, &a);
    if (abs_sum) *abs_sum = fabs(P->scale) * a;
    return P->scale * v;
}

static double orc_entry_q(const orc_problem *P, const __float128 g[6], int i, int j, int p, int q,
                          int r, double *abs_sum)
{
    double bd[6];
    orc_corners(P, i, j, p, q, r, bd); /* exact: coordinates are sums of exact binaries */
    if (P->kind == 2) { if (abs_sum) *abs_sum = 0; return orc_probe_value(P, bd, r); }
    __float128 b[6], a = 0;
    for (int t = 0; t < 6; ++t) b[t] = bd[t];
    /* recompute the corners in quad from the integer indices so that no
     * double rounding enters the coordinates */
    __float128 ai = ((__float128)i + 0.5Q) * P->dx, bj = ((__float128)j + 0.5Q) * P->dy;
    __float128 x0 = (__float128)(p - P->pxl) * P->dx, y0 = (__float128)(q - P->pyl) * P->dy;
    b[0] = x0 - ai;
    b[1] = x0 + P->dx - ai;
    b[2] = y0 - bj;
    b[3] = y0 + P->dy - bj;
    b[4] = (__float128)P->zedge[r] + P->h;
    b[5] = (__float128)P->zedge[r + 1] + P->h;
    __float128 v = orc_prism_q(P->kind, b, g, &a);
    if (abs_sum) *abs_sum = (double)(fabsq((__float128)P->scale) * a);
    return (double)((__float128)P->scale * v);
}

/* ------------------------------------------------------------------------ */
/* Exported entry points                                                     */
/* ------------------------------------------------------------------------ */

/* One arbitrary prism, b = {chi1, chi2, ups1, ups2, zeta1, zeta2} relative to
 * the station; returns scale * (signed corner sum).  quad != 0 evaluates in
 * __float128 and rounds once.  Used by the pins on the closed forms. */
double orc_prism_value(int kind, const double *b, double incl, double decl, const double *w6, double scale,
                       int quad, double *abs_sum)
{
    double a = 0;
    if (quad) {
        __float128 bq[6], gq[6] = {0, 0, 0, 0, 0, 0}, aq = 0;
        for (int t = 0; t < 6; ++t) bq[t] = b[t];
        if (kind == 1) orc_mag_weights_q(incl, decl, gq);
        if (kind == 3) for (int t = 0; t < 6; ++t) gq[t] = w6[t];
        __float128 v = orc_prism_q(kind, bq, gq, &aq);
        if (abs_sum) *abs_sum = (double)(fabsq((__float128)scale) * aq);
        return (double)((__float128)scale * v);
    }
    double g[6] = {0, 0, 0, 0, 0, 0};
    if (kind == 1) orc_mag_weights_d(incl, decl, g);
    if (kind == 3) for (int t = 0; t < 6; ++t) g[t] = w6[t];
    double v = orc_prism_d(kind, b, g, &a);
    if (abs_sum) *abs_sum = fabs(scale) * a;
    return scale * v;
}

/* Dense G (m x n, row-major), every entry from the geometry in double. */
int orc_dense_G(const orc_problem *P, double *G)
{
    const int nx = orc_nx(P), ny = orc_ny(P);
    const int64_t n = (int64_t)nx * ny * P->nz;
    double g[6];
    orc_weights_d(P, g);
#pragma omp parallel for schedule(dynamic, 1)
    for (int k = 0; k < P->sx * P->sy; ++k) {
        const int i = k % P->sx, j = k / P->sx;
        double *row = G + (int64_t)k * n;
        for (int r = 0; r < P->nz; ++r)
            for (int q = 0; q < ny; ++q)
                for (int p = 0; p < nx; ++p)
                    row[(int64_t)r * nx * ny + (int64_t)q * nx + p] =
                        orc_entry_d(P, g, i, j, p, q, r, NULL);
    }
    return 0;
}

/* One entry G[(i,j),(p,q,r)] in double or __float128 (rounded once). */
double orc_entry(const orc_problem *P, int i, int j, int p, int q, int r, int quad, double *abs_sum)
{
    if (quad) {
        __float128 g[6];
        orc_weights_q(P, g);
        return orc_entry_q(P, g, i, j, p, q, r, abs_sum);
    }
    double g[6];
    orc_weights_d(P, g);
    return orc_entry_d(P, g, i, j, p, q, r, abs_sum);
}

/*
 * Entries of G evaluated in __float128 for every (station, prism) pair of the
 * problem, at one representative pair per distinct offset.  The kernels are
 * spatially invariant (Sec. 2.1: h(a,b,c,x,y,z) = h(x-a, y-b, z-c)), so an
 * entry depends only on (p - pxl - i, q - pyl - j, r); the representative pair
 * is chosen with the station inside the data grid and the prism inside the
 * volume.  Output table[r][oy][ox], ox = p - pxl - i + (sx - 1 + pxl) in
 * [0, sx + nx - 1), oy likewise; abs_table holds sum |corner term| * |scale|.
 */
int orc_offset_table_quad(const orc_problem *P, double *table, double *abs_table)
{
    const int nx = orc_nx(P), ny = orc_ny(P);
    const int wx = P->sx + nx - 1, wy = P->sy + ny - 1;
    __float128 g[6];
    orc_weights_q(P, g);
    const int64_t per = (int64_t)wx * wy;
#pragma omp parallel for collapse(2) schedule(dynamic, 4)
    for (int r = 0; r < P->nz; ++r)
        for (int oy = 0; oy < wy; ++oy)
            for (int ox = 0; ox < wx; ++ox) {
                const int dxo = ox - (P->sx - 1 + P->pxl); /* p - pxl - i */
                const int dyo = oy - (P->sy - 1 + P->pyl);
                /* representative: smallest valid station index */
                int i = 0, p = dxo + P->pxl + i;
                if (p < 0) { i = -p; p = 0; }
                int j = 0, q = dyo + P->pyl + j;
                if (q < 0) { j = -q; q = 0; }
                double a = 0;
                double v = orc_entry_q(P, g, i, j, p, q, r, &a);
                table[r * per + (int64_t)oy * wx + ox] = v;
                if (abs_table) abs_table[r * per + (int64_t)oy * wx + ox] = a;
            }
    return 0;
}

/*
 * Direct forward sums d[k] = sum_l G[k][l] m[l] at a list of stations,
 * without forming G.  Following the paper's evaluation of one station's row
 * (Algorithm gravity / Algorithm magnetic, Sec. 4.1): the corner term is
 * evaluated once on the grid of prism edges (x edges 0..nx, y edges 0..ny) for
 * each depth edge, and an entry is the signed sum of its 8 corner values.
 * Sums are accumulated in long double.  m is [nz][ny][nx] (x fastest).
 */
int orc_station_sums(const orc_problem *P, const double *m, int ns, const int32_t *ij, double *out)
{
    const int nx = orc_nx(P), ny = orc_ny(P);
    double g[6];
    orc_weights_d(P, g);
    const int64_t ce = (int64_t)(nx + 1) * (ny + 1);
    double *lo = (double *)malloc(sizeof(double) * ce);
    double *hi = (double *)malloc(sizeof(double) * ce);
    if (!lo || !hi) { free(lo); free(hi); return 1; }
    for (int s = 0; s < ns; ++s) {
        const int i = ij[2 * s], j = ij[2 * s + 1];
        const double a = (i + 0.5) * P->dx, bb = (j + 0.5) * P->dy;
        long double acc = 0;
        for (int r = 0; r < P->nz; ++r) {
            if (P->kind == 2) {
                for (int q = 0; q < ny; ++q)
                    for (int p = 0; p < nx; ++p) {
                        double v = orc_entry_d(P, g, i, j, p, q, r, NULL);
                        acc += (long double)v * m[(int64_t)r * nx * ny + (int64_t)q * nx + p];
                    }
                continue;
            }
            /* corner values at depth edges r (lo) and r+1 (hi) */
            for (int half = 0; half < 2; ++half) {
                double *dst = half ? hi : lo;
                if (half == 0 && r > 0) { memcpy(lo, hi, sizeof(double) * ce); continue; }
                const double zeta = P->zedge[r + half] + P->h;
#pragma omp parallel for schedule(static)
                for (int f = 0; f <= ny; ++f) {
                    const double ups = (f - P->pyl) * P->dy - bb;
                    for (int e = 0; e <= nx; ++e) {
                        const double chi = (e - P->pxl) * P->dx - a;
                        dst[(int64_t)f * (nx + 1) + e] = orc_corner_d(P->kind, chi, ups, zeta, g);
                    }
                }
            }
            long double lacc = 0;
#pragma omp parallel for schedule(static) reduction(+ : lacc)
            for (int q = 0; q < ny; ++q) {
                for (int p = 0; p < nx; ++p) {
                    const int64_t c00 = (int64_t)q * (nx + 1) + p, c01 = c00 + 1;
                    const int64_t c10 = c00 + (nx + 1), c11 = c10 + 1;
                    /* sign (-1)^(i+j+k), index 1 = lower edge: the (lower,lower,lower)
                     * corner carries -1 */
                    double sum = -lo[c00] + lo[c01] + lo[c10] - lo[c11]
                                 + hi[c00] - hi[c01] - hi[c10] + hi[c11];
                    lacc += (long double)(P->scale * sum) *
                            m[(int64_t)r * nx * ny + (int64_t)q * nx + p];
                }
            }
            acc += lacc;
        }
        out[s] = (double)acc;
    }
    free(lo);
    free(hi);
    return 0;
}

/*
 * Direct transpose sums out[l] = sum_k G[k][l] v[k] at a list of prisms
 * (p, q, r), every entry from the geometry (no corner sharing).  v is
 * [sy][sx].  long double accumulation.
 */
int orc_prism_sums(const orc_problem *P, const double *v, int np, const int32_t *pqr, double *out)
{
    double g[6];
    orc_weights_d(P, g);
    for (int s = 0; s < np; ++s) {
        const int p = pqr[3 * s], q = pqr[3 * s + 1], r = pqr[3 * s + 2];
        long double acc = 0;
#pragma omp parallel for schedule(static) reduction(+ : acc)
        for (int j = 0; j < P->sy; ++j) {
            long double a2 = 0;
            for (int i = 0; i < P->sx; ++i)
                a2 += (long double)orc_entry_d(P, g, i, j, p, q, r, NULL) * v[(int64_t)j * P->sx + i];
            acc += a2;
        }
        out[s] = (double)acc;
    }
    return 0;
}

/*
 * The same direct sums with every corner term, entry and partial sum in
 * __float128, rounded to double once at the end: the exact reference for
 * sampled outputs of volumes too large for a dense matrix.  Partial sums are
 * kept per row of the corner grid (per station row for prisms) and added in
 * row order, so the result does not depend on the thread count.
 */
int orc_station_sums_quad(const orc_problem *P, const double *m, int ns, const int32_t *ij, double *out)
{
    const int nx = orc_nx(P), ny = orc_ny(P);
    if (P->kind == 2) return 2;
    __float128 g[6];
    orc_weights_q(P, g);
    const int64_t ce = (int64_t)(nx + 1) * (ny + 1);
    __float128 *lo = (__float128 *)malloc(sizeof(__float128) * ce);
    __float128 *hi = (__float128 *)malloc(sizeof(__float128) * ce);
    __float128 *part = (__float128 *)malloc(sizeof(__float128) * ny);
    if (!lo || !hi || !part) { free(lo); free(hi); free(part); return 1; }
    const __float128 scale = P->scale;
    for (int s = 0; s < ns; ++s) {
        const int i = ij[2 * s], j = ij[2 * s + 1];
        const __float128 a = ((__float128)i + 0.5Q) * P->dx, bb = ((__float128)j + 0.5Q) * P->dy;
        __float128 acc = 0;
        for (int r = 0; r < P->nz; ++r) {
            for (int half = 0; half < 2; ++half) {
                __float128 *dst = half ? hi : lo;
                if (half == 0 && r > 0) { memcpy(lo, hi, sizeof(__float128) * ce); continue; }
                const __float128 zeta = (__float128)P->zedge[r + half] + P->h;
#pragma omp parallel for schedule(dynamic, 4)
                for (int f = 0; f <= ny; ++f) {
                    const __float128 ups = (__float128)(f - P->pyl) * P->dy - bb;
                    for (int e = 0; e <= nx; ++e) {
                        const __float128 chi = (__float128)(e - P->pxl) * P->dx - a;
                        dst[(int64_t)f * (nx + 1) + e] = orc_corner_q(P->kind, chi, ups, zeta, g);
                    }
                }
            }
#pragma omp parallel for schedule(static)
            for (int q = 0; q < ny; ++q) {
                __float128 rowsum = 0;
                for (int p = 0; p < nx; ++p) {
                    const int64_t c00 = (int64_t)q * (nx + 1) + p, c01 = c00 + 1;
                    const int64_t c10 = c00 + (nx + 1), c11 = c10 + 1;
                    const __float128 sum = -lo[c00] + lo[c01] + lo[c10] - lo[c11]
                                           + hi[c00] - hi[c01] - hi[c10] + hi[c11];
                    rowsum += scale * sum * (__float128)m[(int64_t)r * nx * ny + (int64_t)q * nx + p];
                }
                part[q] = rowsum;
            }
            for (int q = 0; q < ny; ++q) acc += part[q];
        }
        out[s] = (double)acc;
    }
    free(lo);
    free(hi);
    free(part);
    return 0;
}

int orc_prism_sums_quad(const orc_problem *P, const double *v, int np, const int32_t *pqr, double *out)
{
    if (P->kind == 2) return 2;
    __float128 g[6];
    orc_weights_q(P, g);
    __float128 *part = (__float128 *)malloc(sizeof(__float128) * P->sy);
    if (!part) return 1;
    for (int s = 0; s < np; ++s) {
        const int p = pqr[3 * s], q = pqr[3 * s + 1], r = pqr[3 * s + 2];
#pragma omp parallel for schedule(dynamic, 4)
        for (int j = 0; j < P->sy; ++j) {
            __float128 rowsum = 0;
            for (int i = 0; i < P->sx; ++i) {
                const __float128 bj = ((__float128)j + 0.5Q) * P->dy, ai = ((__float128)i + 0.5Q) * P->dx;
                const __float128 x0 = (__float128)(p - P->pxl) * P->dx, y0 = (__float128)(q - P->pyl) * P->dy;
                __float128 b[6];
                b[0] = x0 - ai;
                b[1] = x0 + P->dx - ai;
                b[2] = y0 - bj;
                b[3] = y0 + P->dy - bj;
                b[4] = (__float128)P->zedge[r] + P->h;
                b[5] = (__float128)P->zedge[r + 1] + P->h;
                rowsum += (__float128)P->scale * orc_prism_q(P->kind, b, g, NULL) *
                          (__float128)v[(int64_t)j * P->sx + i];
            }
            part[j] = rowsum;
        }
        __float128 acc = 0;
        for (int j = 0; j < P->sy; ++j) acc += part[j];
        out[s] = (double)acc;
    }
    free(part);
    return 0;
}
