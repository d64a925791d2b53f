/*
 * oracle.c -- plain FP64 CPU reference for the horizontal-diffusion +
 * vertical-advection stencil program.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may link, load or
 * call this file: only the tests, the smoke check and the benchmark's CPU
 * baseline leg use it.  It shares no code, header or constant with the HIP
 * library.
 *
 * The paper (Open Earth Compiler, arXiv 2005.13014) optimises stencil
 * programs by inlining (producer-consumer fusion, Sec. V-A) and unrolling
 * (Sec. V-A); both change *where* values are computed, not *what*.  So this
 * oracle is the plain, un-fused definition of each stencil operator of the
 * program, evaluated stage by stage over its full domain, with every
 * temporary materialised in memory (the "original" optimisation level of
 * Sec. VII-C).  Loops are in the literal order of each definition, in
 * double precision, compiled without FP contraction.
 *
 * Array convention (all arrays): dense C order (k, j, i), i fastest, with a
 * halo of width h on both sides in i and j and none in k.  Interior point
 * (i, j, k), 0 <= i < ni, 0 <= j < nj, 0 <= k < nk, lives at
 *     p[((size_t)k * (nj + 2h) + (j + h)) * (ni + 2h) + (i + h)].
 * Negative indices and indices >= n address the halo (the paper's absolute
 * range notation with the origin at the first interior point, Sec. IV-B).
 *
 * "Extension" e: operators write their result on the interior grown by e
 * cells in i and j ([-e, n+e)); inputs must then carry the halo the operator
 * reads (the access extents that shape inference derives, Sec. V-B).
 *
 * Threads: the forward stages carry OpenMP pragmas on their outermost
 * loop (levels for the horizontal stages, rows of columns for the column
 * stages).  Every element is still computed by one thread with the same
 * operations in the same order, so the results are bitwise the same for any
 * thread count; built without -fopenmp (the default) the pragmas are ignored.
 *
 * Readings where the paper is silent (it names these benchmarks but prints
 * no formula):
 *  - hdiff: lap = 4u - u(i+1) - u(i-1) - u(j+1) - u(j-1);
 *    flx = lap(i+1) - lap(i), set to 0 when flx * (u(i+1) - u(i)) > 0
 *    (strictly; a zero product keeps the flux), fly likewise in j;
 *    out = u - coeff * (flx - flx(i-1) + fly - fly(j-1)).
 *  - vertical advection: tridiagonal system a(k) x(k-1) + b(k) x(k)
 *    + c(k) x(k+1) = d(k) per column, solved by the Thomas algorithm (the
 *    implicit vertical integration mentioned in Sec. VII-B); a(0) and
 *    c(nk-1) are ignored.  Right-hand side in flux form:
 *    F(k+1/2) = (w(k)+w(k+1))/2 * (h(k)+h(k+1))/2 for 0 <= k < nk-1,
 *    F(-1/2) = F(nk-1/2) = 0, d(k) = h(k) - dt * (F(k+1/2) - F(k-1/2)).
 *  - vertical diffusion: y(k) = x(k) + kappa * (G(k+1/2) - G(k-1/2)),
 *    G(k+1/2) = x(k+1) - x(k), G(-1/2) = G(nk-1/2) = 0.
 *  - horizontal-gradient update: z = y - bh * ((y(i+1) - y(i-1)) / 2
 *    + (y(j+1) - y(j-1)) / 2) - bv * Dk y, with Dk y = (y(k+1) - y(k-1)) / 2
 *    inside and one-sided differences at the bottom and top levels.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define OK 0
#define ERR_ARG 1
#define ERR_MEM 2

/* Element address in a padded array with halo h. */
static size_t idx(int ni, int nj, int h, int i, int j, int k)
{
    return ((size_t)k * (size_t)(nj + 2 * h) + (size_t)(j + h)) * (size_t)(ni + 2 * h)
           + (size_t)(i + h);
}

static size_t padded_size(int ni, int nj, int nk, int h)
{
    return (size_t)nk * (size_t)(nj + 2 * h) * (size_t)(ni + 2 * h);
}

static int bad_dims(int ni, int nj, int nk)
{
    return ni < 0 || nj < 0 || nk < 0;
}

/* ------------------------------------------------------------------------ */
/* Horizontal diffusion: Laplacian -> limited fluxes -> update.             */
/* ------------------------------------------------------------------------ */

/* Laplacian stage on [-e, ni+e) x [-e, nj+e) for every level.
 * Reads u on the cross (i,j), (i+-1,j), (i,j+-1): needs hu >= e + 1. */
int oracle_lap(int ni, int nj, int nk, const double *u, int hu, double *lap, int hl, int e)
{
    if (bad_dims(ni, nj, nk) || e < 0 || hu < e + 1 || hl < e) return ERR_ARG;
#pragma omp parallel for schedule(static)
    for (int k = 0; k < nk; ++k)
        for (int j = -e; j < nj + e; ++j)
            for (int i = -e; i < ni + e; ++i) {
                double v = 4.0 * u[idx(ni, nj, hu, i, j, k)];
                v = v - u[idx(ni, nj, hu, i + 1, j, k)];
                v = v - u[idx(ni, nj, hu, i - 1, j, k)];
                v = v - u[idx(ni, nj, hu, i, j + 1, k)];
                v = v - u[idx(ni, nj, hu, i, j - 1, k)];
                lap[idx(ni, nj, hl, i, j, k)] = v;
            }
    return OK;
}

/* Flux stage in i.  flx(i) = lap(i+1) - lap(i) for i in [-1-e, ni+e-1],
 * j in [-e, nj+e); limited: zeroed when flx * (u(i+1) - u(i)) > 0.
 * kept[] (optional, same layout as flx) records 1 when the raw flux survives.
 * If force_kept is given it replaces the limiter decision (used to evaluate
 * the adjoint under a mask taken elsewhere). */
static void flux_i(int ni, int nj, int nk, const double *u, int hu, const double *lap, int hl,
                   double *flx, int hf, unsigned char *kept, const unsigned char *force_kept, int e)
{
#pragma omp parallel for schedule(static)
    for (int k = 0; k < nk; ++k)
        for (int j = -e; j < nj + e; ++j)
            for (int i = -1 - e; i < ni + e; ++i) {
                size_t fi = idx(ni, nj, hf, i, j, k);
                double f = lap[idx(ni, nj, hl, i + 1, j, k)] - lap[idx(ni, nj, hl, i, j, k)];
                double du = u[idx(ni, nj, hu, i + 1, j, k)] - u[idx(ni, nj, hu, i, j, k)];
                int keep = force_kept ? (force_kept[fi] != 0) : !(f * du > 0.0);
                flx[fi] = keep ? f : 0.0;
                if (kept) kept[fi] = (unsigned char)keep;
            }
}

/* Flux stage in j, same definition with the roles of i and j swapped:
 * fly(j) = lap(j+1) - lap(j) for j in [-1-e, nj+e-1], i in [-e, ni+e). */
static void flux_j(int ni, int nj, int nk, const double *u, int hu, const double *lap, int hl,
                   double *fly, int hf, unsigned char *kept, const unsigned char *force_kept, int e)
{
#pragma omp parallel for schedule(static)
    for (int k = 0; k < nk; ++k)
        for (int j = -1 - e; j < nj + e; ++j)
            for (int i = -e; i < ni + e; ++i) {
                size_t fi = idx(ni, nj, hf, i, j, k);
                double f = lap[idx(ni, nj, hl, i, j + 1, k)] - lap[idx(ni, nj, hl, i, j, k)];
                double du = u[idx(ni, nj, hu, i, j + 1, k)] - u[idx(ni, nj, hu, i, j, k)];
                int keep = force_kept ? (force_kept[fi] != 0) : !(f * du > 0.0);
                fly[fi] = keep ? f : 0.0;
                if (kept) kept[fi] = (unsigned char)keep;
            }
}

/* Full horizontal diffusion on [-e, ni+e) x [-e, nj+e).
 * u needs halo hu >= e + 2 (13-point diamond); coeff halo hc >= e; out halo ho >= e.
 * Optional outputs (NULL to skip), all with halo e + 1 so that every flux fits:
 *   flx_out/fly_out: the effective (limited) fluxes,
 *   kx/ky: 1 where the raw flux was kept, 0 where the limiter zeroed it.
 * Optional inputs force_kx/force_ky (halo e + 1) override the limiter decision. */
int oracle_hdiff_ex(int ni, int nj, int nk, const double *u, int hu, const double *coeff, int hc,
                    double *out, int ho, int e, double *flx_out, double *fly_out, unsigned char *kx,
                    unsigned char *ky, const unsigned char *force_kx, const unsigned char *force_ky)
{
    if (bad_dims(ni, nj, nk) || e < 0 || hu < e + 2 || hc < e || ho < e) return ERR_ARG;
    int hl = e + 1, hf = e + 1;
    size_t n = padded_size(ni, nj, nk, hl);
    double *lap = (double *)calloc(n ? n : 1, sizeof(double));
    double *flx = (double *)calloc(n ? n : 1, sizeof(double));
    double *fly = (double *)calloc(n ? n : 1, sizeof(double));
    if (!lap || !flx || !fly) {
        free(lap); free(flx); free(fly);
        return ERR_MEM;
    }
    /* lap on [-e-1, n+e+1): the extent the flux stage reads. */
    oracle_lap(ni, nj, nk, u, hu, lap, hl, e + 1);
    flux_i(ni, nj, nk, u, hu, lap, hl, flx, hf, kx, force_kx, e);
    flux_j(ni, nj, nk, u, hu, lap, hl, fly, hf, ky, force_ky, e);
#pragma omp parallel for schedule(static)
    for (int k = 0; k < nk; ++k)
        for (int j = -e; j < nj + e; ++j)
            for (int i = -e; i < ni + e; ++i) {
                double div = flx[idx(ni, nj, hf, i, j, k)] - flx[idx(ni, nj, hf, i - 1, j, k)]
                             + fly[idx(ni, nj, hf, i, j, k)] - fly[idx(ni, nj, hf, i, j - 1, k)];
                out[idx(ni, nj, ho, i, j, k)] =
                    u[idx(ni, nj, hu, i, j, k)] - coeff[idx(ni, nj, hc, i, j, k)] * div;
            }
    if (flx_out) memcpy(flx_out, flx, n * sizeof(double));
    if (fly_out) memcpy(fly_out, fly, n * sizeof(double));
    free(lap); free(flx); free(fly);
    return OK;
}

int oracle_hdiff(int ni, int nj, int nk, const double *u, int hu, const double *coeff, int hc,
                 double *out, int ho, int e)
{
    return oracle_hdiff_ex(ni, nj, nk, u, hu, coeff, hc, out, ho, e, NULL, NULL, NULL, NULL, NULL,
                           NULL);
}

/* ------------------------------------------------------------------------ */
/* Vertical advection: flux-form right-hand side + Thomas solve.            */
/* ------------------------------------------------------------------------ */

/* d(k) = h(k) - dt * (F(k+1/2) - F(k-1/2)) with zero flux through the bottom
 * and top faces.  Column-local: every input needs halo >= e. */
int oracle_rhs(int ni, int nj, int nk, const double *h, int hh, const double *w, int hw, double dt,
               double *d, int hd, int e)
{
    if (bad_dims(ni, nj, nk) || e < 0 || hh < e || hw < e || hd < e) return ERR_ARG;
#pragma omp parallel for schedule(static)
    for (int j = -e; j < nj + e; ++j)
        for (int i = -e; i < ni + e; ++i)
            for (int k = 0; k < nk; ++k) {
                double f_up = 0.0, f_dn = 0.0;
                if (k + 1 < nk) {
                    double wf = 0.5 * (w[idx(ni, nj, hw, i, j, k)] + w[idx(ni, nj, hw, i, j, k + 1)]);
                    double hf = 0.5 * (h[idx(ni, nj, hh, i, j, k)] + h[idx(ni, nj, hh, i, j, k + 1)]);
                    f_up = wf * hf;
                }
                if (k > 0) {
                    double wf = 0.5 * (w[idx(ni, nj, hw, i, j, k - 1)] + w[idx(ni, nj, hw, i, j, k)]);
                    double hf = 0.5 * (h[idx(ni, nj, hh, i, j, k - 1)] + h[idx(ni, nj, hh, i, j, k)]);
                    f_dn = wf * hf;
                }
                d[idx(ni, nj, hd, i, j, k)] = h[idx(ni, nj, hh, i, j, k)] - dt * (f_up - f_dn);
            }
    return OK;
}

/* Thomas algorithm on one column given as strided views.
 * Forward elimination: c'(0) = c(0)/b(0), d'(0) = d(0)/b(0);
 *   m = b(k) - a(k) c'(k-1), c'(k) = c(k)/m, d'(k) = (d(k) - a(k) d'(k-1))/m.
 * Back substitution: x(n-1) = d'(n-1), x(k) = d'(k) - c'(k) x(k+1).
 * sub(k) multiplies x(k-1), sup(k) multiplies x(k+1); sub(0), sup(n-1) unused. */
static void thomas_column(int n, const double *sub, const double *diag, const double *sup,
                          const double *rhs, size_t stride, double *x, double *cp, double *dp)
{
    for (int k = 0; k < n; ++k) {
        size_t o = (size_t)k * stride;
        if (k == 0) {
            cp[0] = (n > 1 ? sup[o] : 0.0) / diag[o];
            dp[0] = rhs[o] / diag[o];
        } else {
            double m = diag[o] - sub[o] * cp[k - 1];
            cp[k] = (k + 1 < n ? sup[o] : 0.0) / m;
            dp[k] = (rhs[o] - sub[o] * dp[k - 1]) / m;
        }
    }
    for (int k = n - 1; k >= 0; --k) {
        size_t o = (size_t)k * stride;
        x[o] = (k == n - 1) ? dp[k] : dp[k] - cp[k] * x[o + stride];
    }
}

/* Solve T x = d per column, T = tridiag(a, b, c) along k. */
int oracle_thomas(int ni, int nj, int nk, const double *a, int ha, const double *b, int hb,
                  const double *c, int hc, const double *d, int hd, double *x, int hx, int e)
{
    if (bad_dims(ni, nj, nk) || e < 0 || ha < e || hb < e || hc < e || hd < e || hx < e)
        return ERR_ARG;
    if (nk == 0) return OK;
    int failed = 0;
#pragma omp parallel for schedule(static) reduction(| : failed)
    for (int j = -e; j < nj + e; ++j) {
        /* The column walker below needs one layout; copy each column out. */
        double *col = (double *)malloc((size_t)nk * 7 * sizeof(double));
        if (!col) {
            failed = 1;
            continue;
        }
        double *ca = col, *cb = col + nk, *cc = col + 2 * nk, *cd = col + 3 * nk, *cx = col + 4 * nk,
               *cp = col + 5 * nk, *dp = col + 6 * nk;
        for (int i = -e; i < ni + e; ++i) {
            for (int k = 0; k < nk; ++k) {
                ca[k] = a[idx(ni, nj, ha, i, j, k)];
                cb[k] = b[idx(ni, nj, hb, i, j, k)];
                cc[k] = c[idx(ni, nj, hc, i, j, k)];
                cd[k] = d[idx(ni, nj, hd, i, j, k)];
            }
            thomas_column(nk, ca, cb, cc, cd, 1, cx, cp, dp);
            for (int k = 0; k < nk; ++k) x[idx(ni, nj, hx, i, j, k)] = cx[k];
        }
        free(col);
    }
    return failed ? ERR_MEM : OK;
}

/* Transposed solve T^T lam = g per column.  T^T has sub-diagonal c(k-1),
 * diagonal b(k), super-diagonal a(k+1); the entries a(0) and c(nk-1) of T
 * are structurally zero and never read. */
int oracle_thomas_transpose(int ni, int nj, int nk, const double *a, int ha, const double *b,
                            int hb, const double *c, int hc, const double *g, int hg, double *lam,
                            int hl, int e)
{
    if (bad_dims(ni, nj, nk) || e < 0 || ha < e || hb < e || hc < e || hg < e || hl < e)
        return ERR_ARG;
    if (nk == 0) return OK;
    double *col = (double *)malloc((size_t)nk * 7 * sizeof(double));
    if (!col) return ERR_MEM;
    double *tsub = col, *tdiag = col + nk, *tsup = col + 2 * nk, *cg = col + 3 * nk,
           *cl = col + 4 * nk, *cp = col + 5 * nk, *dp = col + 6 * nk;
    for (int j = -e; j < nj + e; ++j)
        for (int i = -e; i < ni + e; ++i) {
            for (int k = 0; k < nk; ++k) {
                tsub[k] = k > 0 ? c[idx(ni, nj, hc, i, j, k - 1)] : 0.0;
                tdiag[k] = b[idx(ni, nj, hb, i, j, k)];
                tsup[k] = k + 1 < nk ? a[idx(ni, nj, ha, i, j, k + 1)] : 0.0;
                cg[k] = g[idx(ni, nj, hg, i, j, k)];
            }
            thomas_column(nk, tsub, tdiag, tsup, cg, 1, cl, cp, dp);
            for (int k = 0; k < nk; ++k) lam[idx(ni, nj, hl, i, j, k)] = cl[k];
        }
    free(col);
    return OK;
}

/* vadv = Thomas(a, b, c, rhs(h, w, dt)). */
int oracle_vadv(int ni, int nj, int nk, const double *h, int hh, const double *w, int hw,
                const double *a, int ha, const double *b, int hb, const double *c, int hc,
                double dt, double *x, int hx, int e)
{
    if (bad_dims(ni, nj, nk) || e < 0) return ERR_ARG;
    size_t n = padded_size(ni, nj, nk, e);
    double *d = (double *)malloc((n ? n : 1) * sizeof(double));
    if (!d) return ERR_MEM;
    int rc = oracle_rhs(ni, nj, nk, h, hh, w, hw, dt, d, e, e);
    if (rc == OK) rc = oracle_thomas(ni, nj, nk, a, ha, b, hb, c, hc, d, e, x, hx, e);
    free(d);
    return rc;
}

/* The fused program of the hot path: x = vadv(hdiff(u, coeff), wcon, a, b, c, dt).
 * Materialises h in memory (no fusion). */
int oracle_hdiff_vadv(int ni, int nj, int nk, const double *u, int hu, const double *coeff,
                      int hcf, const double *w, int hw, const double *a, int ha, const double *b,
                      int hb, const double *c, int hc, double dt, double *x, int hx, int e)
{
    if (bad_dims(ni, nj, nk) || e < 0) return ERR_ARG;
    size_t n = padded_size(ni, nj, nk, e);
    double *h = (double *)malloc((n ? n : 1) * sizeof(double));
    if (!h) return ERR_MEM;
    int rc = oracle_hdiff(ni, nj, nk, u, hu, coeff, hcf, h, e, e);
    if (rc == OK) rc = oracle_vadv(ni, nj, nk, h, e, w, hw, a, ha, b, hb, c, hc, dt, x, hx, e);
    free(h);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Stages of the batched timestep.                                          */
/* ------------------------------------------------------------------------ */

/* 3-point vertical diffusion with zero-flux bottom and top faces. */
int oracle_vdiff(int ni, int nj, int nk, const double *x, int hx, double kappa, double *y, int hy,
                 int e)
{
    if (bad_dims(ni, nj, nk) || e < 0 || hx < e || hy < e) return ERR_ARG;
#pragma omp parallel for schedule(static)
    for (int k = 0; k < nk; ++k)
        for (int j = -e; j < nj + e; ++j)
            for (int i = -e; i < ni + e; ++i) {
                double g_up = k + 1 < nk
                                  ? x[idx(ni, nj, hx, i, j, k + 1)] - x[idx(ni, nj, hx, i, j, k)]
                                  : 0.0;
                double g_dn = k > 0 ? x[idx(ni, nj, hx, i, j, k)] - x[idx(ni, nj, hx, i, j, k - 1)]
                                    : 0.0;
                y[idx(ni, nj, hy, i, j, k)] = x[idx(ni, nj, hx, i, j, k)] + kappa * (g_up - g_dn);
            }
    return OK;
}

/* Implicit (backward-Euler) 3-point vertical diffusion with zero-flux bottom
 * and top faces: y solves y(k) - kappa (G(k+1/2) - G(k-1/2)) = x(k) with
 * G(k+1/2) = y(k+1) - y(k) inside the column and G = 0 through its two end
 * faces, i.e. the tridiagonal system -kappa y(k-1) + (1 + 2 kappa) y(k)
 * - kappa y(k+1) = x(k) whose end rows lose the kappa of the missing face.
 * Solved per column by the Thomas algorithm. */
int oracle_vdiff_implicit(int ni, int nj, int nk, const double *x, int hx, double kappa, double *y,
                          int hy, int e)
{
    if (bad_dims(ni, nj, nk) || e < 0 || hx < e || hy < e) return ERR_ARG;
    if (nk == 0) return OK;
    double *col = (double *)malloc((size_t)nk * 7 * sizeof(double));
    if (!col) return ERR_MEM;
    double *sub = col, *diag = col + nk, *sup = col + 2 * nk, *rhs = col + 3 * nk, *out = col + 4 * nk;
    double *cp = col + 5 * nk, *dp = col + 6 * nk;
    for (int k = 0; k < nk; ++k) {
        sub[k] = k > 0 ? -kappa : 0.0;
        sup[k] = k + 1 < nk ? -kappa : 0.0;
        diag[k] = 1.0 + (k > 0 ? kappa : 0.0) + (k + 1 < nk ? kappa : 0.0);
    }
    for (int j = -e; j < nj + e; ++j)
        for (int i = -e; i < ni + e; ++i) {
            for (int k = 0; k < nk; ++k) rhs[k] = x[idx(ni, nj, hx, i, j, k)];
            thomas_column(nk, sub, diag, sup, rhs, 1, out, cp, dp);
            for (int k = 0; k < nk; ++k) y[idx(ni, nj, hy, i, j, k)] = out[k];
        }
    free(col);
    return OK;
}

/* 7-point horizontal-gradient update: centred differences in i and j, centred
 * in k inside the column and one-sided at its two ends.  Needs hy >= e + 1. */
int oracle_hgrad(int ni, int nj, int nk, const double *y, int hy, double beta_h, double beta_v,
                 double *z, int hz, int e)
{
    if (bad_dims(ni, nj, nk) || e < 0 || hy < e + 1 || hz < e) return ERR_ARG;
#pragma omp parallel for schedule(static)
    for (int k = 0; k < nk; ++k)
        for (int j = -e; j < nj + e; ++j)
            for (int i = -e; i < ni + e; ++i) {
                double gi = 0.5 * (y[idx(ni, nj, hy, i + 1, j, k)] - y[idx(ni, nj, hy, i - 1, j, k)]);
                double gj = 0.5 * (y[idx(ni, nj, hy, i, j + 1, k)] - y[idx(ni, nj, hy, i, j - 1, k)]);
                double gk;
                if (nk == 1)
                    gk = 0.0;
                else if (k == 0)
                    gk = y[idx(ni, nj, hy, i, j, 1)] - y[idx(ni, nj, hy, i, j, 0)];
                else if (k == nk - 1)
                    gk = y[idx(ni, nj, hy, i, j, nk - 1)] - y[idx(ni, nj, hy, i, j, nk - 2)];
                else
                    gk = 0.5 * (y[idx(ni, nj, hy, i, j, k + 1)] - y[idx(ni, nj, hy, i, j, k - 1)]);
                z[idx(ni, nj, hz, i, j, k)] =
                    y[idx(ni, nj, hy, i, j, k)] - beta_h * (gi + gj) - beta_v * gk;
            }
    return OK;
}

/* One field of the batched timestep: hdiff -> vadv -> vdiff on the interior
 * grown by one cell (the ring hgrad reads), then hgrad on the interior.
 * implicit != 0 takes the implicit vertical diffusion.
 * u needs halo >= 3, the coefficient fields halo >= 1. */
int oracle_timestep_ex(int ni, int nj, int nk, const double *u, int hu, const double *coeff, int hcf,
                       const double *w, int hw, const double *a, int ha, const double *b, int hb,
                       const double *c, int hc, double dt, double kappa, double beta_h,
                       double beta_v, int implicit, double *z, int hz)
{
    if (bad_dims(ni, nj, nk)) return ERR_ARG;
    size_t n = padded_size(ni, nj, nk, 1);
    double *x = (double *)malloc((n ? n : 1) * sizeof(double));
    double *y = (double *)malloc((n ? n : 1) * sizeof(double));
    if (!x || !y) {
        free(x); free(y);
        return ERR_MEM;
    }
    int rc = oracle_hdiff_vadv(ni, nj, nk, u, hu, coeff, hcf, w, hw, a, ha, b, hb, c, hc, dt, x, 1, 1);
    if (rc == OK)
        rc = implicit ? oracle_vdiff_implicit(ni, nj, nk, x, 1, kappa, y, 1, 1)
                      : oracle_vdiff(ni, nj, nk, x, 1, kappa, y, 1, 1);
    if (rc == OK) rc = oracle_hgrad(ni, nj, nk, y, 1, beta_h, beta_v, z, hz, 0);
    free(x); free(y);
    return rc;
}

int oracle_timestep(int ni, int nj, int nk, const double *u, int hu, const double *coeff, int hcf,
                    const double *w, int hw, const double *a, int ha, const double *b, int hb,
                    const double *c, int hc, double dt, double kappa, double beta_h, double beta_v,
                    double *z, int hz)
{
    return oracle_timestep_ex(ni, nj, nk, u, hu, coeff, hcf, w, hw, a, ha, b, hb, c, hc, dt, kappa,
                              beta_h, beta_v, 0, z, hz);
}

/* ------------------------------------------------------------------------ */
/* Reverse mode (adjoint) of x = vadv(hdiff(u, coeff), wcon, a, b, c, dt).  */
/* ------------------------------------------------------------------------ */

/* Adjoint of the right-hand side.  Given lam = dL/dd, accumulates
 *   gh(k) = lam(k) + sum over faces f touching k of 1/2 * Fhat(f) * wbar(f),
 *   gw(k) =          sum over faces f touching k of 1/2 * Fhat(f) * hbar(f),
 * where Fhat(k+1/2) = -dt * (lam(k) - lam(k+1)), wbar, hbar the face means.
 * gh and gw are overwritten on the interior. */
int oracle_rhs_adjoint(int ni, int nj, int nk, const double *h, int hh, const double *w, int hw,
                       double dt, const double *lam, int hl, double *gh, int hgh, double *gw,
                       int hgw)
{
    if (bad_dims(ni, nj, nk)) return ERR_ARG;
    for (int j = 0; j < nj; ++j)
        for (int i = 0; i < ni; ++i) {
            for (int k = 0; k < nk; ++k) {
                gh[idx(ni, nj, hgh, i, j, k)] = lam[idx(ni, nj, hl, i, j, k)];
                gw[idx(ni, nj, hgw, i, j, k)] = 0.0;
            }
            for (int k = 0; k + 1 < nk; ++k) {
                double fhat = -dt * (lam[idx(ni, nj, hl, i, j, k)] - lam[idx(ni, nj, hl, i, j, k + 1)]);
                double wbar = 0.5 * (w[idx(ni, nj, hw, i, j, k)] + w[idx(ni, nj, hw, i, j, k + 1)]);
                double hbar = 0.5 * (h[idx(ni, nj, hh, i, j, k)] + h[idx(ni, nj, hh, i, j, k + 1)]);
                gh[idx(ni, nj, hgh, i, j, k)] += 0.5 * fhat * wbar;
                gh[idx(ni, nj, hgh, i, j, k + 1)] += 0.5 * fhat * wbar;
                gw[idx(ni, nj, hgw, i, j, k)] += 0.5 * fhat * hbar;
                gw[idx(ni, nj, hgw, i, j, k + 1)] += 0.5 * fhat * hbar;
            }
        }
    return OK;
}

/* Adjoint of hdiff on the interior, limiter decisions frozen (the derivative
 * of the 0/1 mask is taken as zero).  gh: dL/dh on the interior.  Outputs:
 * gu (halo >= 2; interior and 2-cell ring written, overwritten) and gcoeff
 * (interior, overwritten).  force_kx/ky (halo 1, optional) replace the
 * limiter decisions; otherwise they are recomputed from u. */
int oracle_hdiff_adjoint(int ni, int nj, int nk, const double *u, int hu, const double *coeff,
                         int hc, const double *gh, int hgh, double *gu, int hgu, double *gcoeff,
                         int hgc, const unsigned char *force_kx, const unsigned char *force_ky)
{
    if (bad_dims(ni, nj, nk) || hu < 2 || hgu < 2) return ERR_ARG;
    size_t n1 = padded_size(ni, nj, nk, 1);
    double *flx = (double *)calloc(n1 ? n1 : 1, sizeof(double));
    double *fly = (double *)calloc(n1 ? n1 : 1, sizeof(double));
    unsigned char *kx = (unsigned char *)calloc(n1 ? n1 : 1, 1);
    unsigned char *ky = (unsigned char *)calloc(n1 ? n1 : 1, 1);
    double *gfx = (double *)calloc(n1 ? n1 : 1, sizeof(double));
    double *gfy = (double *)calloc(n1 ? n1 : 1, sizeof(double));
    double *glap = (double *)calloc(n1 ? n1 : 1, sizeof(double));
    double *hbuf = (double *)calloc(padded_size(ni, nj, nk, 0) + 1, sizeof(double));
    if (!flx || !fly || !kx || !ky || !gfx || !gfy || !glap || !hbuf) {
        free(flx); free(fly); free(kx); free(ky); free(gfx); free(gfy); free(glap); free(hbuf);
        return ERR_MEM;
    }
    /* Forward recomputation of the fluxes and of the limiter decisions. */
    oracle_hdiff_ex(ni, nj, nk, u, hu, coeff, hc, hbuf, 0, 0, flx, fly, kx, ky, force_kx, force_ky);

    for (size_t q = 0; q < padded_size(ni, nj, nk, hgu); ++q) gu[q] = 0.0;

    /* Update stage: h = u - coeff * (flx(i) - flx(i-1) + fly(j) - fly(j-1)). */
    for (int k = 0; k < nk; ++k)
        for (int j = 0; j < nj; ++j)
            for (int i = 0; i < ni; ++i) {
                double g = gh[idx(ni, nj, hgh, i, j, k)];
                double div = flx[idx(ni, nj, 1, i, j, k)] - flx[idx(ni, nj, 1, i - 1, j, k)]
                             + fly[idx(ni, nj, 1, i, j, k)] - fly[idx(ni, nj, 1, i, j - 1, k)];
                gcoeff[idx(ni, nj, hgc, i, j, k)] = -g * div;
                gu[idx(ni, nj, hgu, i, j, k)] += g;
                double gdiv = -coeff[idx(ni, nj, hc, i, j, k)] * g;
                gfx[idx(ni, nj, 1, i, j, k)] += gdiv;
                gfx[idx(ni, nj, 1, i - 1, j, k)] -= gdiv;
                gfy[idx(ni, nj, 1, i, j, k)] += gdiv;
                gfy[idx(ni, nj, 1, i, j - 1, k)] -= gdiv;
            }
    /* Flux stages: flx(i) = mask * (lap(i+1) - lap(i)); likewise fly. */
    for (int k = 0; k < nk; ++k)
        for (int j = 0; j < nj; ++j)
            for (int i = -1; i < ni; ++i) {
                size_t fi = idx(ni, nj, 1, i, j, k);
                double g = kx[fi] ? gfx[fi] : 0.0;
                glap[idx(ni, nj, 1, i + 1, j, k)] += g;
                glap[idx(ni, nj, 1, i, j, k)] -= g;
            }
    for (int k = 0; k < nk; ++k)
        for (int j = -1; j < nj; ++j)
            for (int i = 0; i < ni; ++i) {
                size_t fi = idx(ni, nj, 1, i, j, k);
                double g = ky[fi] ? gfy[fi] : 0.0;
                glap[idx(ni, nj, 1, i, j + 1, k)] += g;
                glap[idx(ni, nj, 1, i, j, k)] -= g;
            }
    /* Laplacian stage: lap = 4u - u(i+1) - u(i-1) - u(j+1) - u(j-1) on [-1, n]. */
    for (int k = 0; k < nk; ++k)
        for (int j = -1; j <= nj; ++j)
            for (int i = -1; i <= ni; ++i) {
                double g = glap[idx(ni, nj, 1, i, j, k)];
                gu[idx(ni, nj, hgu, i, j, k)] += 4.0 * g;
                gu[idx(ni, nj, hgu, i + 1, j, k)] -= g;
                gu[idx(ni, nj, hgu, i - 1, j, k)] -= g;
                gu[idx(ni, nj, hgu, i, j + 1, k)] -= g;
                gu[idx(ni, nj, hgu, i, j - 1, k)] -= g;
            }
    free(flx); free(fly); free(kx); free(ky); free(gfx); free(gfy); free(glap); free(hbuf);
    return OK;
}

/* Gradient of L = sum over the interior of wl * x, x = vadv(hdiff(u, coeff)),
 * with respect to u (interior + 2-cell ring), coeff and wcon (interior).
 * ga, gb, gc (optional, NULL to skip): gradients with respect to the matrix
 * entries, -lam(k) x(k-1), -lam(k) x(k), -lam(k) x(k+1) (zero where the entry
 * is structurally absent).  force_kx/ky as in oracle_hdiff_adjoint. */
int oracle_hdiff_vadv_adjoint(int ni, int nj, int nk, const double *u, int hu,
                              const double *coeff, int hcf, const double *w, int hw,
                              const double *a, int ha, const double *b, int hb, const double *c,
                              int hc, double dt, const double *wl, int hwl, double *gu, int hgu,
                              double *gcoeff, int hgc, double *gw, int hgw, double *ga, double *gb,
                              double *gc, int hgm, const unsigned char *force_kx,
                              const unsigned char *force_ky)
{
    if (bad_dims(ni, nj, nk) || hu < 2 || hgu < 2) return ERR_ARG;
    size_t n = padded_size(ni, nj, nk, 0);
    double *h = (double *)malloc((n + 1) * sizeof(double));
    double *lam = (double *)malloc((n + 1) * sizeof(double));
    double *gh = (double *)malloc((n + 1) * sizeof(double));
    double *x = (double *)malloc((n + 1) * sizeof(double));
    if (!h || !lam || !gh || !x) {
        free(h); free(lam); free(gh); free(x);
        return ERR_MEM;
    }
    int rc = oracle_hdiff_ex(ni, nj, nk, u, hu, coeff, hcf, h, 0, 0, NULL, NULL, NULL, NULL,
                             force_kx, force_ky);
    if (rc == OK) rc = oracle_thomas_transpose(ni, nj, nk, a, ha, b, hb, c, hc, wl, hwl, lam, 0, 0);
    if (rc == OK) rc = oracle_rhs_adjoint(ni, nj, nk, h, 0, w, hw, dt, lam, 0, gh, 0, gw, hgw);
    if (rc == OK)
        rc = oracle_hdiff_adjoint(ni, nj, nk, u, hu, coeff, hcf, gh, 0, gu, hgu, gcoeff, hgc,
                                  force_kx, force_ky);
    if (rc == OK && (ga || gb || gc)) {
        rc = oracle_vadv(ni, nj, nk, h, 0, w, hw, a, ha, b, hb, c, hc, dt, x, 0, 0);
        for (int k = 0; rc == OK && k < nk; ++k)
            for (int j = 0; j < nj; ++j)
                for (int i = 0; i < ni; ++i) {
                    double l = lam[idx(ni, nj, 0, i, j, k)];
                    size_t o = idx(ni, nj, hgm, i, j, k);
                    if (ga) ga[o] = k > 0 ? -l * x[idx(ni, nj, 0, i, j, k - 1)] : 0.0;
                    if (gb) gb[o] = -l * x[idx(ni, nj, 0, i, j, k)];
                    if (gc) gc[o] = k + 1 < nk ? -l * x[idx(ni, nj, 0, i, j, k + 1)] : 0.0;
                }
    }
    free(h); free(lam); free(gh); free(x);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Forward mode: the tangent of x = hdiff_vadv(u, coeff, w, a, b, c).       */
/* ------------------------------------------------------------------------ */

/* Tangent of the flux-form right-hand side: with F(k+1/2) = wf * hf (the two
 * face averages), dF = (dw face average) * hf + wf * (dh face average), and
 * dd(k) = dh(k) - dt * (dF(k+1/2) - dF(k-1/2)), zero tangent flux through the
 * bottom and top faces.  dw may be NULL (zero).  All arrays on the interior. */
static void rhs_tangent(int ni, int nj, int nk, const double *h, const double *dh, const double *w,
                        int hw, const double *dw, int hdw, double dt, double *dd)
{
    for (int j = 0; j < nj; ++j)
        for (int i = 0; i < ni; ++i)
            for (int k = 0; k < nk; ++k) {
                double df[2] = {0.0, 0.0}; /* below, above */
                for (int s = 0; s < 2; ++s) {
                    int k0 = s ? k : k - 1, k1 = k0 + 1;
                    if (k0 < 0 || k1 >= nk) continue;
                    double wf = 0.5 * (w[idx(ni, nj, hw, i, j, k0)] + w[idx(ni, nj, hw, i, j, k1)]);
                    double hf = 0.5 * (h[idx(ni, nj, 0, i, j, k0)] + h[idx(ni, nj, 0, i, j, k1)]);
                    double dwf = dw ? 0.5 * (dw[idx(ni, nj, hdw, i, j, k0)] + dw[idx(ni, nj, hdw, i, j, k1)])
                                    : 0.0;
                    double dhf = 0.5 * (dh[idx(ni, nj, 0, i, j, k0)] + dh[idx(ni, nj, 0, i, j, k1)]);
                    df[s] = dwf * hf + wf * dhf;
                }
                dd[idx(ni, nj, 0, i, j, k)] = dh[idx(ni, nj, 0, i, j, k)] - dt * (df[1] - df[0]);
            }
}

/* dx = J v for the direction v = (du, dcoeff, dw, da, db, dc); any of them
 * may be NULL (a zero tangent).  The limiter masks are those of the forward
 * pass (or force_kx / force_ky): the operator is piecewise linear in u on
 * each side of a limiter switch, and the tangent is the derivative of the
 * piece the forward pass took.  Stages, each the derivative of its forward
 * counterpart:
 *   dlap = lap(du); dflx = kept ? dlap(i+1) - dlap(i) : 0 (dfly likewise);
 *   dh = du - dcoeff * div - coeff * ddiv, div and ddiv the flux divergences;
 *   dd = tangent of the right-hand side (rhs_tangent);
 *   T dx = dd - (da x(k-1) + db x(k) + dc x(k+1)), x the forward solution,
 * the last because T x = d gives dT x + T dx = dd.  du needs halo 2 like u;
 * dx is written on the interior with halo hdx. */
int oracle_hdiff_vadv_jvp(int ni, int nj, int nk, const double *u, int hu, const double *coeff,
                          int hcf, const double *w, int hw, const double *a, int ha, const double *b,
                          int hb, const double *c, int hc, double dt, const double *du, int hdu,
                          const double *dcoeff, int hdcf, const double *dw, int hdw, const double *da,
                          const double *db, const double *dc, int hdm, double *dx, int hdx,
                          const unsigned char *force_kx, const unsigned char *force_ky)
{
    if (bad_dims(ni, nj, nk) || hu < 2 || hcf < 0 || hw < 0 || ha < 0 || hb < 0 || hc < 0 ||
        (du && hdu < 2) || hdcf < 0 || hdw < 0 || hdm < 0 || hdx < 0)
        return ERR_ARG;
    size_t n = padded_size(ni, nj, nk, 0), n1 = padded_size(ni, nj, nk, 1);
    double *h = (double *)malloc((n + 1) * sizeof(double));
    double *x = (double *)malloc((n + 1) * sizeof(double));
    double *dh = (double *)calloc(n + 1, sizeof(double));
    double *dd = (double *)malloc((n + 1) * sizeof(double));
    double *flx = (double *)calloc(n1 + 1, sizeof(double));
    double *fly = (double *)calloc(n1 + 1, sizeof(double));
    double *dlap = (double *)calloc(n1 + 1, sizeof(double));
    double *dflx = (double *)calloc(n1 + 1, sizeof(double));
    double *dfly = (double *)calloc(n1 + 1, sizeof(double));
    unsigned char *kx = (unsigned char *)calloc(n1 + 1, 1);
    unsigned char *ky = (unsigned char *)calloc(n1 + 1, 1);
    int rc = OK;
    if (!h || !x || !dh || !dd || !flx || !fly || !dlap || !dflx || !dfly || !kx || !ky) rc = ERR_MEM;
    /* Forward pass: h with its limited fluxes and keep masks, then x. */
    if (rc == OK)
        rc = oracle_hdiff_ex(ni, nj, nk, u, hu, coeff, hcf, h, 0, 0, flx, fly, kx, ky, force_kx,
                             force_ky);
    if (rc == OK) rc = oracle_vadv(ni, nj, nk, h, 0, w, hw, a, ha, b, hb, c, hc, dt, x, 0, 0);
    /* Tangent of hdiff under the forward masks. */
    if (rc == OK && du) {
        rc = oracle_lap(ni, nj, nk, du, hdu, dlap, 1, 1);
        if (rc == OK) {
            flux_i(ni, nj, nk, du, hdu, dlap, 1, dflx, 1, NULL, kx, 0);
            flux_j(ni, nj, nk, du, hdu, dlap, 1, dfly, 1, NULL, ky, 0);
        }
    }
    for (int k = 0; rc == OK && k < nk; ++k)
        for (int j = 0; j < nj; ++j)
            for (int i = 0; i < ni; ++i) {
                double div = flx[idx(ni, nj, 1, i, j, k)] - flx[idx(ni, nj, 1, i - 1, j, k)]
                             + fly[idx(ni, nj, 1, i, j, k)] - fly[idx(ni, nj, 1, i, j - 1, k)];
                double ddiv = dflx[idx(ni, nj, 1, i, j, k)] - dflx[idx(ni, nj, 1, i - 1, j, k)]
                              + dfly[idx(ni, nj, 1, i, j, k)] - dfly[idx(ni, nj, 1, i, j - 1, k)];
                double v = du ? du[idx(ni, nj, hdu, i, j, k)] : 0.0;
                if (dcoeff) v -= dcoeff[idx(ni, nj, hdcf, i, j, k)] * div;
                v -= coeff[idx(ni, nj, hcf, i, j, k)] * ddiv;
                dh[idx(ni, nj, 0, i, j, k)] = v;
            }
    /* Tangent of the right-hand side, minus the matrix tangent applied to x. */
    if (rc == OK) {
        rhs_tangent(ni, nj, nk, h, dh, w, hw, dw, hdw, dt, dd);
        for (int k = 0; k < nk; ++k)
            for (int j = 0; j < nj; ++j)
                for (int i = 0; i < ni; ++i) {
                    double r = dd[idx(ni, nj, 0, i, j, k)];
                    if (da && k > 0) r -= da[idx(ni, nj, hdm, i, j, k)] * x[idx(ni, nj, 0, i, j, k - 1)];
                    if (db) r -= db[idx(ni, nj, hdm, i, j, k)] * x[idx(ni, nj, 0, i, j, k)];
                    if (dc && k + 1 < nk) r -= dc[idx(ni, nj, hdm, i, j, k)] * x[idx(ni, nj, 0, i, j, k + 1)];
                    dd[idx(ni, nj, 0, i, j, k)] = r;
                }
        rc = oracle_thomas(ni, nj, nk, a, ha, b, hb, c, hc, dd, 0, dx, hdx, 0);
    }
    free(h); free(x); free(dh); free(dd); free(flx); free(fly); free(dlap); free(dflx); free(dfly);
    free(kx); free(ky);
    return rc;
}
