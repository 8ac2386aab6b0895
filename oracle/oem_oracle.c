/*
 * OEM oracle: plain FP64 CPU reference.  TEST INFRASTRUCTURE ONLY: used by
 * the test suite, the smoke check and the benchmark's CPU baseline, never by
 * the product library.  See oem_oracle.h for the problem statement.
 *
 * Built with -O2 -ffp-contract=off: every multiply and add is rounded as
 * written.
 */
#include "oem_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Fold assignment                                                           */
/* ------------------------------------------------------------------------ */

/* SplitMix64 as published by Steele, Lea & Flood (2014): a Weyl sequence with
 * increment 0x9E3779B97F4A7C15 passed through a variant of the MurmurHash3
 * 64-bit finaliser. */
uint64_t oracle_splitmix64_next(uint64_t *state)
{
    *state += 0x9E3779B97F4A7C15ULL;
    uint64_t z = *state;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* Section 3 partitions the rows at random into K folds.  Row i takes the
 * (i+1)-th SplitMix64 output from state = seed; the fold is
 * floor(K * hi32 / 2^32). */
int32_t oracle_fold_of_row(uint64_t seed, int64_t i, int32_t K)
{
    uint64_t state = seed + (uint64_t)i * 0x9E3779B97F4A7C15ULL;
    uint64_t r = oracle_splitmix64_next(&state);
    uint64_t hi = r >> 32;
    return (int32_t)((hi * (uint64_t)K) >> 32);
}

static int32_t row_fold(int64_t i, int64_t row_offset, int32_t K, uint64_t seed,
                        const uint8_t *foldid)
{
    if (K == 1) return 0;
    if (foldid) return (int32_t)foldid[i];
    return oracle_fold_of_row(seed, row_offset + i, K);
}

static double x_at(const void *X, int32_t x_is_f64, int64_t ldx, int64_t i, int32_t j)
{
    if (x_is_f64) return ((const double *)X)[i * ldx + j];
    return (double)((const float *)X)[i * ldx + j];
}

/* ------------------------------------------------------------------------ */
/* Sufficient statistics (Section 3)                                          */
/* ------------------------------------------------------------------------ */

int oracle_gram_folds(const void *X, int32_t x_is_f64, int64_t n, int64_t ldx, int32_t p,
                      const double *y, int64_t row_offset, int32_t K, uint64_t fold_seed,
                      const uint8_t *foldid, double *G, double *b, double *yy, int64_t *nk)
{
    if (p <= 0 || K <= 0 || n < 0 || ldx < p) return -1;
    memset(G, 0, sizeof(double) * (size_t)K * p * p);
    memset(b, 0, sizeof(double) * (size_t)K * p);
    memset(yy, 0, sizeof(double) * (size_t)K);
    memset(nk, 0, sizeof(int64_t) * (size_t)K);
    for (int64_t i = 0; i < n; ++i) {
        int32_t k = row_fold(i, row_offset, K, fold_seed, foldid);
        if (k < 0 || k >= K) return -1;
        double *Gk = G + (size_t)k * p * p;
        for (int32_t a = 0; a < p; ++a) {
            double xa = x_at(X, x_is_f64, ldx, i, a);
            for (int32_t c = 0; c < p; ++c)
                Gk[(size_t)a * p + c] += xa * x_at(X, x_is_f64, ldx, i, c);
            b[(size_t)k * p + a] += xa * y[i];
        }
        yy[k] += y[i] * y[i];
        nk[k] += 1;
    }
    return 0;
}

int oracle_gram_csr(const int64_t *rowptr, const int32_t *col, const double *val, int64_t n, int32_t p,
                    const double *y, int64_t row_offset, int32_t K, uint64_t fold_seed,
                    const uint8_t *foldid, double *G, double *b, double *yy, int64_t *nk)
{
    if (p <= 0 || K <= 0 || n < 0) return -1;
    memset(G, 0, sizeof(double) * (size_t)K * p * p);
    memset(b, 0, sizeof(double) * (size_t)K * p);
    memset(yy, 0, sizeof(double) * (size_t)K);
    memset(nk, 0, sizeof(int64_t) * (size_t)K);
    for (int64_t i = 0; i < n; ++i) {
        int32_t k = row_fold(i, row_offset, K, fold_seed, foldid);
        if (k < 0 || k >= K || rowptr[i] > rowptr[i + 1]) return -1;
        double *Gk = G + (size_t)k * p * p;
        for (int64_t t = rowptr[i]; t < rowptr[i + 1]; ++t) {
            if (col[t] < 0 || col[t] >= p) return -1;
            for (int64_t u = rowptr[i]; u < rowptr[i + 1]; ++u)
                Gk[(size_t)col[t] * p + col[u]] += val[t] * val[u];
            b[(size_t)k * p + col[t]] += val[t] * y[i];
        }
        yy[k] += y[i] * y[i];
        nk[k] += 1;
    }
    return 0;
}

int oracle_gram_train(const void *X, int32_t x_is_f64, int64_t n, int64_t ldx, int32_t p,
                      const double *y, int64_t row_offset, int32_t K, uint64_t fold_seed,
                      const uint8_t *foldid, int32_t k, double *G, double *b, double *yy,
                      int64_t *ntrain)
{
    if (p <= 0 || K <= 0 || n < 0 || ldx < p) return -1;
    memset(G, 0, sizeof(double) * (size_t)p * p);
    memset(b, 0, sizeof(double) * (size_t)p);
    *yy = 0.0;
    *ntrain = 0;
    for (int64_t i = 0; i < n; ++i) {
        if (k >= 0 && row_fold(i, row_offset, K, fold_seed, foldid) == k) continue;
        for (int32_t a = 0; a < p; ++a) {
            double xa = x_at(X, x_is_f64, ldx, i, a);
            for (int32_t c = 0; c < p; ++c)
                G[(size_t)a * p + c] += xa * x_at(X, x_is_f64, ldx, i, c);
            b[a] += xa * y[i];
        }
        *yy += y[i] * y[i];
        *ntrain += 1;
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Standardisation (Section 2.1 assumes unit-norm columns)                    */
/* ------------------------------------------------------------------------ */

void oracle_standardize(int32_t p, const double *G, const double *c, double *Gs, double *cs,
                        double *s)
{
    for (int32_t j = 0; j < p; ++j) {
        double gjj = G[(size_t)j * p + j];
        s[j] = gjj > 0.0 ? sqrt(gjj) : 1.0;
    }
    for (int32_t a = 0; a < p; ++a) {
        for (int32_t b2 = 0; b2 < p; ++b2)
            Gs[(size_t)a * p + b2] = G[(size_t)a * p + b2] / (s[a] * s[b2]);
        cs[a] = c[a] / s[a];
    }
}

/* ------------------------------------------------------------------------ */
/* Largest eigenvalue (Section 2.1: d >= lambda_1, d = lambda_1 fastest)     */
/* ------------------------------------------------------------------------ */

/* Cyclic Jacobi: sweep over every off-diagonal pair (q, r), q < r, and apply
 * the plane rotation that zeroes A_qr.  For a rotation with cosine c and sine
 * s, t = s/c is the smaller root of t^2 + 2 theta t - 1 = 0 where
 * theta = (A_rr - A_qq) / (2 A_qr).  Stops when the off-diagonal Frobenius
 * norm is negligible next to the diagonal. */
int oracle_sym_eigvals(int32_t p, const double *A, double *eig)
{
    double *a = (double *)malloc(sizeof(double) * (size_t)p * p);
    if (!a) return -1;
    memcpy(a, A, sizeof(double) * (size_t)p * p);
    int sweeps = -1;
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0, diag = 0.0;
        for (int32_t q = 0; q < p; ++q)
            for (int32_t r = 0; r < p; ++r) {
                double v = a[(size_t)q * p + r];
                if (q == r) diag += v * v;
                else off += v * v;
            }
        if (off <= 1e-36 * diag || off == 0.0) { sweeps = sweep; break; }
        for (int32_t q = 0; q < p - 1; ++q) {
            for (int32_t r = q + 1; r < p; ++r) {
                double aqr = a[(size_t)q * p + r];
                if (aqr == 0.0) continue;
                double aqq = a[(size_t)q * p + q], arr = a[(size_t)r * p + r];
                double theta = (arr - aqq) / (2.0 * aqr);
                double t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
                double c = 1.0 / sqrt(t * t + 1.0);
                double s = t * c;
                /* A <- J^T A J with J the rotation in the (q, r) plane. */
                for (int32_t m = 0; m < p; ++m) {
                    double amq = a[(size_t)m * p + q], amr = a[(size_t)m * p + r];
                    a[(size_t)m * p + q] = c * amq - s * amr;
                    a[(size_t)m * p + r] = s * amq + c * amr;
                }
                for (int32_t m = 0; m < p; ++m) {
                    double aqm = a[(size_t)q * p + m], arm = a[(size_t)r * p + m];
                    a[(size_t)q * p + m] = c * aqm - s * arm;
                    a[(size_t)r * p + m] = s * aqm + c * arm;
                }
                a[(size_t)q * p + r] = 0.0;
                a[(size_t)r * p + q] = 0.0;
            }
        }
    }
    for (int32_t j = 0; j < p; ++j) eig[j] = a[(size_t)j * p + j];
    free(a);
    return sweeps;
}

double oracle_oem_d(int32_t p, const double *A)
{
    double *e = (double *)malloc(sizeof(double) * (size_t)p);
    if (!e) return -1.0;
    if (oracle_sym_eigvals(p, A, e) < 0) { free(e); return -1.0; }
    double m = e[0];
    for (int32_t j = 1; j < p; ++j)
        if (e[j] > m) m = e[j];
    free(e);
    return m * (1.0 + 1e-10);
}

/* ------------------------------------------------------------------------ */
/* Thresholding operators (Section 2.2)                                       */
/* ------------------------------------------------------------------------ */

static double sgn(double v) { return v > 0.0 ? 1.0 : (v < 0.0 ? -1.0 : 0.0); }
static double pos(double v) { return v > 0.0 ? v : 0.0; }

double oracle_prox1(const oracle_penalty *pen, double u, double lam_w, double d)
{
    double au = fabs(u);
    switch (pen->kind) {
    case ORACLE_LASSO: /* eq. (lasso): S(u, w lambda, d) */
        return sgn(u) * pos(au - lam_w) / d;
    case ORACLE_ENET: /* eq. (net) */
        return sgn(u) * pos(au - lam_w * pen->alpha) / (d + lam_w * (1.0 - pen->alpha));
    case ORACLE_MCP: { /* eq. (mcp): M(u, w lambda, gamma, d) */
        double g = pen->gamma;
        if (au <= lam_w * g * d) return sgn(u) * g * pos(au - lam_w) / (g * d - 1.0);
        return u / d;
    }
    case ORACLE_SCAD: { /* eq. (scad): C(u, w lambda, gamma, d) */
        double g = pen->gamma;
        if (au <= (d + 1.0) * lam_w) return sgn(u) * pos(au - lam_w) / d;
        if (au <= lam_w * g * d) return sgn(u) * ((g - 1.0) * au - lam_w * g) / ((g - 1.0) * d - 1.0);
        return u / d;
    }
    default:
        return NAN;
    }
}

/* eq. (glasso): G(u_g, c_k lambda, d) = (u_g / d)(1 - c_k lambda / ||u_g||)_+ */
void oracle_prox_group(int32_t m, const double *u, double lam_c, double d, double *out)
{
    double ss = 0.0;
    for (int32_t j = 0; j < m; ++j) ss += u[j] * u[j];
    double nrm = sqrt(ss);
    double f = nrm > 0.0 ? 1.0 - lam_c / nrm : 0.0;
    for (int32_t j = 0; j < m; ++j) out[j] = f > 0.0 ? (u[j] / d) * f : 0.0;
}

static int is_group_kind(int32_t kind)
{
    return kind == ORACLE_GRP_LASSO || kind == ORACLE_GRP_MCP || kind == ORACLE_GRP_SCAD ||
           kind == ORACLE_SGL;
}

void oracle_prox_group_pen(const oracle_penalty *pen, int32_t m, const double *u, const double *w,
                           double cgk, double lambda, double d, double *out)
{
    if (pen->kind == ORACLE_GRP_LASSO) {
        oracle_prox_group(m, u, cgk * lambda, d, out);
        return;
    }
    if (pen->kind == ORACLE_SGL) {
        /* eq. (sglasso) with the proximal map of the nested penalty taken
         * as written out: inner soft threshold at w_j lambda tau without the
         * 1/d, then G(v, c_k lambda (1 - tau), d). */
        double *v = (double *)malloc(sizeof(double) * (size_t)(m > 0 ? m : 1));
        for (int32_t j = 0; j < m; ++j) {
            double t = (w ? w[j] : 1.0) * lambda * pen->tau;
            v[j] = sgn(u[j]) * pos(fabs(u[j]) - t);
        }
        oracle_prox_group(m, v, cgk * lambda * (1.0 - pen->tau), d, out);
        free(v);
        return;
    }
    /* eqs. (gmcp), (gscad): M or C of ||u|| at c_k lambda, direction u/||u|| */
    double ss = 0.0;
    for (int32_t j = 0; j < m; ++j) ss += u[j] * u[j];
    double nrm = sqrt(ss);
    oracle_penalty scalar = *pen;
    scalar.kind = pen->kind == ORACLE_GRP_MCP ? ORACLE_MCP : ORACLE_SCAD;
    double t = nrm > 0.0 ? oracle_prox1(&scalar, nrm, cgk * lambda, d) : 0.0;
    for (int32_t j = 0; j < m; ++j) out[j] = t > 0.0 ? t * (u[j] / nrm) : 0.0;
}

/* ------------------------------------------------------------------------ */
/* Group bookkeeping                                                          */
/* ------------------------------------------------------------------------ */

typedef struct {
    int32_t ng;
    int32_t *start; /* ng + 1 */
    int32_t *idx;   /* p: variables listed group by group, ascending within */
} groupmap;

static int groupmap_build(int32_t p, const int32_t *groups, int32_t ngroups, groupmap *gm)
{
    gm->ng = ngroups;
    gm->start = (int32_t *)calloc((size_t)ngroups + 1, sizeof(int32_t));
    gm->idx = (int32_t *)malloc(sizeof(int32_t) * (size_t)p);
    if (!gm->start || !gm->idx) return -1;
    for (int32_t j = 0; j < p; ++j) {
        if (groups[j] < 0 || groups[j] >= ngroups) return -1;
        gm->start[groups[j] + 1] += 1;
    }
    for (int32_t g = 0; g < ngroups; ++g) {
        if (gm->start[g + 1] == 0) return -1; /* every group id must be used */
        gm->start[g + 1] += gm->start[g];
    }
    int32_t *fill = (int32_t *)calloc((size_t)ngroups, sizeof(int32_t));
    if (!fill) return -1;
    for (int32_t j = 0; j < p; ++j) {
        int32_t g = groups[j];
        gm->idx[gm->start[g] + fill[g]++] = j;
    }
    free(fill);
    return 0;
}

static void groupmap_free(groupmap *gm)
{
    free(gm->start);
    free(gm->idx);
}

static double w_of(const double *w, int32_t j) { return w ? w[j] : 1.0; }

static double cg_of(const double *cg, const groupmap *gm, int32_t g)
{
    return cg ? cg[g] : sqrt((double)(gm->start[g + 1] - gm->start[g]));
}

/* Apply the penalty's update to the whole vector u. */
static void prox_all(int32_t p, const oracle_penalty *pen, const groupmap *gm, const double *w,
                     const double *cg, double lambda, double d, const double *u, double *out,
                     double *tmp_u, double *tmp_o)
{
    if (is_group_kind(pen->kind)) {
        double *wg = (double *)malloc(sizeof(double) * (size_t)p);
        for (int32_t g = 0; g < gm->ng; ++g) {
            int32_t m = gm->start[g + 1] - gm->start[g];
            for (int32_t t = 0; t < m; ++t) {
                tmp_u[t] = u[gm->idx[gm->start[g] + t]];
                wg[t] = w_of(w, gm->idx[gm->start[g] + t]);
            }
            oracle_prox_group_pen(pen, m, tmp_u, wg, cg_of(cg, gm, g), lambda, d, tmp_o);
            for (int32_t t = 0; t < m; ++t) out[gm->idx[gm->start[g] + t]] = tmp_o[t];
        }
        free(wg);
    } else {
        for (int32_t j = 0; j < p; ++j) out[j] = oracle_prox1(pen, u[j], w_of(w, j) * lambda, d);
    }
}

/* ------------------------------------------------------------------------ */
/* lambda sequence                                                            */
/* ------------------------------------------------------------------------ */

/* Does the sparse group lasso update of group g map beta = 0 (so u = cs) to
 * a nonzero vector at this lambda?  The test is the update's own: inner
 * soft threshold, then the group factor 1 - c_k lambda (1 - tau) / ||v||. */
static int sgl_group_nonzero(const groupmap *gm, int32_t g, const double *cs, const double *w,
                             double cgk, double tau, double lambda)
{
    double ss = 0.0;
    for (int32_t t = gm->start[g]; t < gm->start[g + 1]; ++t) {
        int32_t j = gm->idx[t];
        double v = pos(fabs(cs[j]) - w_of(w, j) * lambda * tau);
        ss += v * v;
    }
    double nrm = sqrt(ss);
    return nrm > 0.0 && 1.0 - cgk * lambda * (1.0 - tau) / nrm > 0.0;
}

/* Smallest lambda at which group g's sparse group lasso update maps beta = 0
 * to 0.  tau = 1 is the lasso: each penalised member's own threshold.
 * Otherwise ||soft(c_g, w lambda tau)|| - c_k lambda (1 - tau) decreases in
 * lambda and is <= 0 at ||c_g|| / (c_k (1 - tau)); the crossing is found by
 * bisection over doubles down to adjacent values. */
static double sgl_group_lambda_max(const groupmap *gm, int32_t g, const double *cs, const double *w,
                                   double cgk, double tau)
{
    if (tau >= 1.0) {
        double lg = 0.0;
        for (int32_t t = gm->start[g]; t < gm->start[g + 1]; ++t) {
            int32_t j = gm->idx[t];
            double wj = w_of(w, j);
            if (wj <= 0.0) continue;
            double lj = fabs(cs[j]) / wj;
            while (fabs(cs[j]) - wj * lj > 0.0) lj = nextafter(lj, INFINITY);
            if (lj > lg) lg = lj;
        }
        return lg;
    }
    double ss = 0.0;
    for (int32_t t = gm->start[g]; t < gm->start[g + 1]; ++t) ss += cs[gm->idx[t]] * cs[gm->idx[t]];
    double lo = 0.0, hi = sqrt(ss) / (cgk * (1.0 - tau));
    if (!sgl_group_nonzero(gm, g, cs, w, cgk, tau, lo)) return 0.0;
    while (sgl_group_nonzero(gm, g, cs, w, cgk, tau, hi)) hi = nextafter(hi, INFINITY);
    for (;;) {
        double mid = lo + 0.5 * (hi - lo);
        if (!(mid > lo && mid < hi)) break;
        if (sgl_group_nonzero(gm, g, cs, w, cgk, tau, mid))
            lo = mid;
        else
            hi = mid;
    }
    return hi;
}

double oracle_lambda_max(int32_t p, const double *cs, const oracle_penalty *pen,
                         const int32_t *groups, int32_t ngroups, const double *w,
                         const double *cg)
{
    double lmax = 0.0;
    if (pen->kind == ORACLE_SGL) {
        groupmap gm;
        if (!groups || groupmap_build(p, groups, ngroups, &gm) != 0) return -1.0;
        for (int32_t g = 0; g < gm.ng; ++g) {
            double lg = sgl_group_lambda_max(&gm, g, cs, w, cg_of(cg, &gm, g), pen->tau);
            if (lg > lmax) lmax = lg;
        }
        groupmap_free(&gm);
        return lmax;
    }
    if (is_group_kind(pen->kind)) {
        groupmap gm;
        if (!groups || groupmap_build(p, groups, ngroups, &gm) != 0) return -1.0;
        for (int32_t g = 0; g < gm.ng; ++g) {
            double ss = 0.0;
            for (int32_t t = gm.start[g]; t < gm.start[g + 1]; ++t) ss += cs[gm.idx[t]] * cs[gm.idx[t]];
            double nrm = sqrt(ss), c = cg_of(cg, &gm, g);
            double lg = nrm / c;
            /* smallest lambda the group update itself maps to zero: the
             * group lasso factor 1 - c lambda / ||u||, or the soft part
             * ||u|| - c lambda of the MCP / SCAD update of ||u|| */
            if (pen->kind == ORACLE_GRP_LASSO)
                while (nrm > 0.0 && 1.0 - c * lg / nrm > 0.0) lg = nextafter(lg, INFINITY);
            else
                while (nrm - c * lg > 0.0) lg = nextafter(lg, INFINITY);
            if (lg > lmax) lmax = lg;
        }
        groupmap_free(&gm);
        return lmax;
    }
    double a = pen->kind == ORACLE_ENET ? pen->alpha : 1.0;
    for (int32_t j = 0; j < p; ++j) {
        double wj = w_of(w, j);
        if (wj <= 0.0) continue; /* unpenalised variable never limits lambda */
        double lj = fabs(cs[j]) / (wj * a);
        if (pen->kind == ORACLE_ENET)
            while (fabs(cs[j]) - wj * lj * a > 0.0) lj = nextafter(lj, INFINITY);
        else
            while (fabs(cs[j]) - wj * lj > 0.0) lj = nextafter(lj, INFINITY);
        if (lj > lmax) lmax = lj;
    }
    return lmax;
}

void oracle_lambda_grid(double lambda_max, int32_t L, double ratio, double *lambda)
{
    for (int32_t l = 0; l < L; ++l)
        lambda[l] = L == 1 ? lambda_max : lambda_max * pow(ratio, (double)l / (double)(L - 1));
}

/* ------------------------------------------------------------------------ */
/* Objective and KKT (standardised problem)                                   */
/* ------------------------------------------------------------------------ */

static double mcp_value(double b, double lw, double g)
{
    double ab = fabs(b);
    return ab <= g * lw ? lw * ab - b * b / (2.0 * g) : 0.5 * g * lw * lw;
}

static double scad_value(double b, double lw, double g)
{
    double ab = fabs(b);
    if (ab <= lw) return lw * ab;
    if (ab <= g * lw) return -(ab * ab - 2.0 * g * lw * ab + lw * lw) / (2.0 * (g - 1.0));
    return 0.5 * (g + 1.0) * lw * lw;
}

static double penalty_value(int32_t p, const oracle_penalty *pen, const groupmap *gm,
                            const double *w, const double *cg, double lambda, const double *beta)
{
    double s = 0.0;
    if (is_group_kind(pen->kind)) {
        /* penalty table; group MCP / SCAD read as sum_k P_{lambda c_k, gamma}(||beta_g||) */
        for (int32_t g = 0; g < gm->ng; ++g) {
            double ss = 0.0, l1 = 0.0;
            for (int32_t t = gm->start[g]; t < gm->start[g + 1]; ++t) {
                ss += beta[gm->idx[t]] * beta[gm->idx[t]];
                l1 += w_of(w, gm->idx[t]) * fabs(beta[gm->idx[t]]);
            }
            double lc = lambda * cg_of(cg, gm, g), bn = sqrt(ss);
            switch (pen->kind) {
            case ORACLE_GRP_LASSO: s += lc * bn; break;
            case ORACLE_GRP_MCP: s += mcp_value(bn, lc, pen->gamma); break;
            case ORACLE_GRP_SCAD: s += scad_value(bn, lc, pen->gamma); break;
            default: s += (1.0 - pen->tau) * lc * bn + pen->tau * lambda * l1; break;
            }
        }
        return s;
    }
    for (int32_t j = 0; j < p; ++j) {
        double lw = lambda * w_of(w, j), b = beta[j];
        switch (pen->kind) {
        case ORACLE_LASSO: s += lw * fabs(b); break;
        case ORACLE_ENET:
            s += pen->alpha * lw * fabs(b) + 0.5 * (1.0 - pen->alpha) * lw * b * b;
            break;
        case ORACLE_MCP: s += mcp_value(b, lw, pen->gamma); break;
        case ORACLE_SCAD: s += scad_value(b, lw, pen->gamma); break;
        default: return NAN;
        }
    }
    return s;
}

static double objective_gm(int32_t p, const double *Gs, const double *cs, double yyn,
                           const oracle_penalty *pen, const groupmap *gm, const double *w,
                           const double *cg, double lambda, const double *beta)
{
    double q = 0.0, l = 0.0;
    for (int32_t a = 0; a < p; ++a) {
        double row = 0.0;
        for (int32_t b2 = 0; b2 < p; ++b2) row += Gs[(size_t)a * p + b2] * beta[b2];
        q += beta[a] * row;
        l += cs[a] * beta[a];
    }
    return 0.5 * q - l + 0.5 * yyn + penalty_value(p, pen, gm, w, cg, lambda, beta);
}

/* Stationarity 0 in grad + dP(beta), grad = Gs beta - cs. */
static double kkt_gm(int32_t p, const double *Gs, const double *cs, const oracle_penalty *pen,
                     const groupmap *gm, const double *w, const double *cg, double lambda,
                     const double *beta)
{
    double *gr = (double *)malloc(sizeof(double) * (size_t)p);
    if (!gr) return NAN;
    for (int32_t a = 0; a < p; ++a) {
        double row = 0.0;
        for (int32_t b2 = 0; b2 < p; ++b2) row += Gs[(size_t)a * p + b2] * beta[b2];
        gr[a] = row - cs[a];
    }
    double viol = 0.0;
    if (pen->kind == ORACLE_SGL) {
        /* 0 in grad_g + lambda (1 - tau) c_k dN(beta_g) + lambda tau w * d|beta_g|,
         * N the Euclidean norm.  Zero group: the distance of -grad_g to the
         * sum of the box and the ball is ||soft(grad_g, lambda tau w)||
         * less the ball radius.  Nonzero group: per member, the residual with
         * the norm's gradient beta_j / ||beta_g||; zero members take the
         * distance of their residual to [-lambda tau w_j, lambda tau w_j]. */
        for (int32_t g = 0; g < gm->ng; ++g) {
            double lc = lambda * (1.0 - pen->tau) * cg_of(cg, gm, g), bn = 0.0;
            for (int32_t t = gm->start[g]; t < gm->start[g + 1]; ++t)
                bn += beta[gm->idx[t]] * beta[gm->idx[t]];
            bn = sqrt(bn);
            double ss = 0.0, v;
            for (int32_t t = gm->start[g]; t < gm->start[g + 1]; ++t) {
                int32_t j = gm->idx[t];
                double lt = lambda * pen->tau * w_of(w, j), r;
                if (bn == 0.0)
                    r = pos(fabs(gr[j]) - lt);
                else if (beta[j] == 0.0)
                    r = pos(fabs(gr[j]) - lt);
                else
                    r = gr[j] + lc * beta[j] / bn + lt * sgn(beta[j]);
                ss += r * r;
            }
            v = bn == 0.0 ? pos(sqrt(ss) - lc) : sqrt(ss);
            if (v > viol) viol = v;
        }
        free(gr);
        return viol;
    }
    if (pen->kind == ORACLE_GRP_MCP || pen->kind == ORACLE_GRP_SCAD) {
        /* 0 in grad_g + P'(||beta_g||) beta_g / ||beta_g|| (nonzero group),
         * ||grad_g|| <= lambda c_k (zero group: P'(0+) = lambda c_k) */
        for (int32_t g = 0; g < gm->ng; ++g) {
            double lc = lambda * cg_of(cg, gm, g), bn = 0.0, gn = 0.0, v;
            for (int32_t t = gm->start[g]; t < gm->start[g + 1]; ++t) {
                bn += beta[gm->idx[t]] * beta[gm->idx[t]];
                gn += gr[gm->idx[t]] * gr[gm->idx[t]];
            }
            bn = sqrt(bn);
            gn = sqrt(gn);
            if (bn > 0.0) {
                double gam = pen->gamma, dp;
                if (pen->kind == ORACLE_GRP_MCP)
                    dp = pos(lc - bn / gam);
                else
                    dp = bn <= lc ? lc : (bn <= gam * lc ? (gam * lc - bn) / (gam - 1.0) : 0.0);
                double ss = 0.0;
                for (int32_t t = gm->start[g]; t < gm->start[g + 1]; ++t) {
                    int32_t j = gm->idx[t];
                    double r = gr[j] + dp * beta[j] / bn;
                    ss += r * r;
                }
                v = sqrt(ss);
            } else {
                v = pos(gn - lc);
            }
            if (v > viol) viol = v;
        }
        free(gr);
        return viol;
    }
    if (pen->kind == ORACLE_GRP_LASSO) {
        for (int32_t g = 0; g < gm->ng; ++g) {
            double lc = lambda * cg_of(cg, gm, g), bn = 0.0, gn = 0.0;
            for (int32_t t = gm->start[g]; t < gm->start[g + 1]; ++t) {
                bn += beta[gm->idx[t]] * beta[gm->idx[t]];
                gn += gr[gm->idx[t]] * gr[gm->idx[t]];
            }
            bn = sqrt(bn);
            gn = sqrt(gn);
            double v;
            if (bn > 0.0) {
                double ss = 0.0;
                for (int32_t t = gm->start[g]; t < gm->start[g + 1]; ++t) {
                    int32_t j = gm->idx[t];
                    double r = gr[j] + lc * beta[j] / bn;
                    ss += r * r;
                }
                v = sqrt(ss);
            } else {
                v = pos(gn - lc);
            }
            if (v > viol) viol = v;
        }
        free(gr);
        return viol;
    }
    for (int32_t j = 0; j < p; ++j) {
        double lw = lambda * w_of(w, j), b = beta[j], ab = fabs(b), v;
        if (b == 0.0) {
            double thr = pen->kind == ORACLE_ENET ? pen->alpha * lw : lw;
            v = pos(fabs(gr[j]) - thr);
        } else {
            double dp; /* derivative of the penalty at |b| */
            switch (pen->kind) {
            case ORACLE_LASSO: dp = lw; break;
            case ORACLE_ENET: dp = pen->alpha * lw + (1.0 - pen->alpha) * lw * ab; break;
            case ORACLE_MCP: dp = pos(lw - ab / pen->gamma); break;
            case ORACLE_SCAD:
                dp = ab <= lw ? lw : (ab <= pen->gamma * lw ? (pen->gamma * lw - ab) / (pen->gamma - 1.0) : 0.0);
                break;
            default: dp = NAN;
            }
            v = fabs(gr[j] + sgn(b) * dp);
        }
        if (v > viol) viol = v;
    }
    free(gr);
    return viol;
}

double oracle_objective(int32_t p, const double *Gs, const double *cs, double yyn,
                        const oracle_penalty *pen, const int32_t *groups, int32_t ngroups,
                        const double *w, const double *cg, double lambda, const double *beta)
{
    groupmap gm = {0, NULL, NULL};
    if (is_group_kind(pen->kind) && (!groups || groupmap_build(p, groups, ngroups, &gm) != 0))
        return NAN;
    double f = objective_gm(p, Gs, cs, yyn, pen, &gm, w, cg, lambda, beta);
    if (is_group_kind(pen->kind)) groupmap_free(&gm);
    return f;
}

double oracle_kkt(int32_t p, const double *Gs, const double *cs, const oracle_penalty *pen,
                  const int32_t *groups, int32_t ngroups, const double *w, const double *cg,
                  double lambda, const double *beta)
{
    groupmap gm = {0, NULL, NULL};
    if (is_group_kind(pen->kind) && (!groups || groupmap_build(p, groups, ngroups, &gm) != 0))
        return NAN;
    double v = kkt_gm(p, Gs, cs, pen, &gm, w, cg, lambda, beta);
    if (is_group_kind(pen->kind)) groupmap_free(&gm);
    return v;
}

/* ------------------------------------------------------------------------ */
/* OEM iterations                                                             */
/* ------------------------------------------------------------------------ */

static int check_penalty(const oracle_penalty *pen, double d)
{
    switch (pen->kind) {
    case ORACLE_LASSO: case ORACLE_GRP_LASSO: return 0;
    case ORACLE_ENET: return (pen->alpha > 0.0 && pen->alpha <= 1.0) ? 0 : -1;
    case ORACLE_MCP: case ORACLE_GRP_MCP: return (pen->gamma > 1.0 && pen->gamma * d > 1.0) ? 0 : -1;
    case ORACLE_SCAD: case ORACLE_GRP_SCAD:
        return (pen->gamma > 2.0 && (pen->gamma - 1.0) * d > 1.0) ? 0 : -1;
    case ORACLE_SGL: return (pen->tau >= 0.0 && pen->tau <= 1.0) ? 0 : -1;
    default: return -1;
    }
}

/* One OEM step (E-step + M-step, Section 2.1): u = cs + (d I - Gs) beta,
 * beta_new = prox(u).  Returns max |beta_new - beta| in *delta and
 * max |beta_new| in *bmax; beta is overwritten with beta_new. */
static void oem_step(int32_t p, const double *Gs, const double *cs, double d,
                     const oracle_penalty *pen, const groupmap *gm, const double *w,
                     const double *cg, double lambda, double *beta, double *u, double *bn,
                     double *tu, double *to, double *delta, double *bmax)
{
    for (int32_t a = 0; a < p; ++a) {
        double gb = 0.0;
        for (int32_t b2 = 0; b2 < p; ++b2) gb += Gs[(size_t)a * p + b2] * beta[b2];
        u[a] = cs[a] + (d * beta[a] - gb);
    }
    prox_all(p, pen, gm, w, cg, lambda, d, u, bn, tu, to);
    double dl = 0.0, mx = 0.0;
    for (int32_t a = 0; a < p; ++a) {
        double df = fabs(bn[a] - beta[a]);
        if (df > dl) dl = df;
        if (fabs(bn[a]) > mx) mx = fabs(bn[a]);
        beta[a] = bn[a];
    }
    *delta = dl;
    *bmax = mx;
}

typedef struct {
    double *u, *bn, *tu, *to;
} scratch;

static int scratch_alloc(int32_t p, scratch *s)
{
    s->u = (double *)malloc(sizeof(double) * (size_t)p);
    s->bn = (double *)malloc(sizeof(double) * (size_t)p);
    s->tu = (double *)malloc(sizeof(double) * (size_t)p);
    s->to = (double *)malloc(sizeof(double) * (size_t)p);
    return (s->u && s->bn && s->tu && s->to) ? 0 : -1;
}

static void scratch_free(scratch *s)
{
    free(s->u); free(s->bn); free(s->tu); free(s->to);
}

int oracle_fit_path(int32_t p, const double *Gs, const double *cs, double yyn, double d,
                    const oracle_penalty *pen, const int32_t *groups, int32_t ngroups,
                    const double *w, const double *cg, int32_t L, const double *lambda,
                    double tol, int32_t maxit, double *beta, int32_t *iters, double *kkt,
                    double *obj)
{
    if (p <= 0 || L < 1 || maxit < 1 || !(d > 0.0) || check_penalty(pen, d) != 0) return -1;
    groupmap gm = {0, NULL, NULL};
    if (is_group_kind(pen->kind) && (!groups || groupmap_build(p, groups, ngroups, &gm) != 0))
        return -1;
    scratch s;
    if (scratch_alloc(p, &s) != 0) return -2;
    double *cur = (double *)calloc((size_t)p, sizeof(double));
    int status = 0;
    for (int32_t l = 0; l < L; ++l) {
        int32_t it = 0, conv = 0;
        while (it < maxit) {
            double dl, mx;
            oem_step(p, Gs, cs, d, pen, &gm, w, cg, lambda[l], cur, s.u, s.bn, s.tu, s.to, &dl, &mx);
            ++it;
            if (dl <= tol * mx) { conv = 1; break; }
        }
        if (!conv) status = 1;
        if (iters) iters[l] = conv ? it : -it;
        memcpy(beta + (size_t)l * p, cur, sizeof(double) * (size_t)p);
        if (kkt) kkt[l] = kkt_gm(p, Gs, cs, pen, &gm, w, cg, lambda[l], cur);
        if (obj) obj[l] = objective_gm(p, Gs, cs, yyn, pen, &gm, w, cg, lambda[l], cur);
    }
    free(cur);
    scratch_free(&s);
    if (is_group_kind(pen->kind)) groupmap_free(&gm);
    return status;
}

int oracle_oem_steps(int32_t p, const double *Gs, const double *cs, double yyn, double d,
                     const oracle_penalty *pen, const int32_t *groups, int32_t ngroups,
                     const double *w, const double *cg, double lambda, int32_t nsteps,
                     double *beta, double *obj_trace)
{
    if (p <= 0 || !(d > 0.0) || check_penalty(pen, d) != 0) return -1;
    groupmap gm = {0, NULL, NULL};
    if (is_group_kind(pen->kind) && (!groups || groupmap_build(p, groups, ngroups, &gm) != 0))
        return -1;
    scratch s;
    if (scratch_alloc(p, &s) != 0) return -2;
    for (int32_t t = 0; t < nsteps; ++t) {
        double dl, mx;
        oem_step(p, Gs, cs, d, pen, &gm, w, cg, lambda, beta, s.u, s.bn, s.tu, s.to, &dl, &mx);
        if (obj_trace) obj_trace[t] = objective_gm(p, Gs, cs, yyn, pen, &gm, w, cg, lambda, beta);
    }
    scratch_free(&s);
    if (is_group_kind(pen->kind)) groupmap_free(&gm);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Cross-validation error from held-out rows                                  */
/* ------------------------------------------------------------------------ */

int oracle_heldout_mse(const void *X, int32_t x_is_f64, int64_t n, int64_t ldx, int32_t p,
                       const double *y, int64_t row_offset, int32_t K, uint64_t fold_seed,
                       const uint8_t *foldid, int32_t k, int32_t L, const double *beta,
                       const double *beta0, double *mse)
{
    if (p <= 0 || L < 1) return -1;
    int64_t nk = 0;
    for (int32_t l = 0; l < L; ++l) mse[l] = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        if (row_fold(i, row_offset, K, fold_seed, foldid) != k) continue;
        ++nk;
        for (int32_t l = 0; l < L; ++l) {
            double pred = beta0 ? beta0[l] : 0.0;
            for (int32_t j = 0; j < p; ++j) pred += x_at(X, x_is_f64, ldx, i, j) * beta[(size_t)l * p + j];
            double r = y[i] - pred;
            mse[l] += r * r;
        }
    }
    if (nk == 0) return -1;
    for (int32_t l = 0; l < L; ++l) mse[l] /= (double)nk;
    return 0;
}

void oracle_fold_ids(uint64_t seed, int64_t row_offset, int64_t n, int32_t K, uint8_t *out)
{
    for (int64_t i = 0; i < n; ++i) out[i] = (uint8_t)oracle_fold_of_row(seed, row_offset + i, K);
}

/* ------------------------------------------------------------------------ */
/* Penalised logistic regression (Section 4)                                  */
/* ------------------------------------------------------------------------ */

/* log(1 + exp(t)) without overflow */
static double softplus(double t) { return t > 0.0 ? t + log1p(exp(-t)) : log1p(exp(t)); }

int oracle_logistic_path(const void *X, int32_t x_is_f64, int64_t n, int64_t ldx, int32_t p,
                         const double *y, const oracle_penalty *pen, const int32_t *groups,
                         int32_t ngroups, const double *w, const double *cg, int32_t L,
                         const double *lambda, int32_t hessian_bound, double tol, int32_t maxit,
                         double newton_tol, int32_t newton_maxit, double *beta, int32_t *newton_iters,
                         double *kkt, double *obj)
{
    if (p <= 0 || n <= 0 || L < 1 || maxit < 1 || newton_maxit < 1) return -1;
    groupmap gm = {0, NULL, NULL};
    if (is_group_kind(pen->kind) && (!groups || groupmap_build(p, groups, ngroups, &gm) != 0)) return -1;
    size_t pp = (size_t)p * p;
    double *s = (double *)calloc((size_t)p, sizeof(double));
    double *H = (double *)malloc(sizeof(double) * pp);
    double *c = (double *)malloc(sizeof(double) * (size_t)p);
    double *bt = (double *)calloc((size_t)p, sizeof(double));   /* standardised coefficients */
    double *prev = (double *)malloc(sizeof(double) * (size_t)p);
    double *eta = (double *)malloc(sizeof(double) * (size_t)n);
    double *wt = (double *)malloc(sizeof(double) * (size_t)n);
    double *z = (double *)malloc(sizeof(double) * (size_t)n);
    double *gr = (double *)malloc(sizeof(double) * (size_t)p);
    scratch sc;
    if (!s || !H || !c || !bt || !prev || !eta || !wt || !z || !gr || scratch_alloc(p, &sc) != 0) return -2;
    /* fixed column scales: unit mean square of each column (Section 2.1) */
    for (int64_t i = 0; i < n; ++i)
        for (int32_t j = 0; j < p; ++j) {
            double v = x_at(X, x_is_f64, ldx, i, j);
            s[j] += v * v;
        }
    for (int32_t j = 0; j < p; ++j) s[j] = s[j] > 0.0 ? sqrt(s[j] / (double)n) : 1.0;
    int status = 0;
    double d = 0.0;
    for (int32_t l = 0; l < L; ++l) {
        int32_t t = 0, conv = 0;
        while (t < newton_maxit) {
            /* working weights and responses at the current coefficients */
            for (int64_t i = 0; i < n; ++i) {
                double e = 0.0;
                for (int32_t j = 0; j < p; ++j) e += x_at(X, x_is_f64, ldx, i, j) * (bt[j] / s[j]);
                double mu = 1.0 / (1.0 + exp(-e));
                eta[i] = e;
                wt[i] = hessian_bound ? 0.25 : mu * (1.0 - mu);
                z[i] = e + (y[i] - mu) / wt[i];
            }
            /* weighted least-squares statistics, standardised */
            if (!hessian_bound || t == 0 || d == 0.0) {
                for (size_t e = 0; e < pp; ++e) H[e] = 0.0;
                for (int64_t i = 0; i < n; ++i) {
                    for (int32_t a = 0; a < p; ++a) gr[a] = x_at(X, x_is_f64, ldx, i, a) / s[a];  /* row i, standardised */
                    for (int32_t a = 0; a < p; ++a)
                        for (int32_t b2 = 0; b2 < p; ++b2) H[(size_t)a * p + b2] += wt[i] * gr[a] * gr[b2];
                }
                for (size_t e = 0; e < pp; ++e) H[e] /= (double)n;
                d = oracle_oem_d(p, H);
            }
            for (int32_t a = 0; a < p; ++a) c[a] = 0.0;
            for (int64_t i = 0; i < n; ++i)
                for (int32_t a = 0; a < p; ++a) c[a] += wt[i] * (x_at(X, x_is_f64, ldx, i, a) / s[a]) * z[i];
            for (int32_t a = 0; a < p; ++a) c[a] /= (double)n;
            /* inner OEM iterations on the quadratic model, from the current point */
            memcpy(prev, bt, sizeof(double) * (size_t)p);
            for (int32_t it = 0; it < maxit; ++it) {
                double dl, mx;
                oem_step(p, H, c, d, pen, &gm, w, cg, lambda[l], bt, sc.u, sc.bn, sc.tu, sc.to, &dl, &mx);
                if (dl <= tol * mx) break;
            }
            ++t;
            double dl = 0.0, mx = 0.0;
            for (int32_t j = 0; j < p; ++j) {
                if (fabs(bt[j] - prev[j]) > dl) dl = fabs(bt[j] - prev[j]);
                if (fabs(bt[j]) > mx) mx = fabs(bt[j]);
            }
            if (dl <= newton_tol * mx) { conv = 1; break; }
        }
        if (!conv) status = 1;
        if (newton_iters) newton_iters[l] = conv ? t : -t;
        for (int32_t j = 0; j < p; ++j) beta[(size_t)l * p + j] = bt[j] / s[j];
        /* objective and stationarity of the logistic problem at the result:
         * gradient of the mean negative log-likelihood, -X~^T (y - mu) / n */
        double loss = 0.0;
        for (int32_t j = 0; j < p; ++j) gr[j] = 0.0;
        for (int64_t i = 0; i < n; ++i) {
            double e = 0.0;
            for (int32_t j = 0; j < p; ++j) e += x_at(X, x_is_f64, ldx, i, j) * (bt[j] / s[j]);
            double mu = 1.0 / (1.0 + exp(-e));
            loss += softplus(e) - y[i] * e;
            for (int32_t j = 0; j < p; ++j) gr[j] -= (x_at(X, x_is_f64, ldx, i, j) / s[j]) * (y[i] - mu);
        }
        for (int32_t j = 0; j < p; ++j) gr[j] /= (double)n;
        if (obj) obj[l] = loss / (double)n + penalty_value(p, pen, &gm, w, cg, lambda[l], bt);
        if (kkt) {
            /* stationarity with Gs = 0 and cs = -gr: the same rules as kkt_gm */
            double *zero = (double *)calloc(pp, sizeof(double));
            for (int32_t j = 0; j < p; ++j) c[j] = -gr[j];
            kkt[l] = kkt_gm(p, zero, c, pen, &gm, w, cg, lambda[l], bt);
            free(zero);
        }
    }
    free(s); free(H); free(c); free(bt); free(prev); free(eta); free(wt); free(z); free(gr);
    scratch_free(&sc);
    if (is_group_kind(pen->kind)) groupmap_free(&gm);
    return status;
}

/* lambda_max of the logistic path: at beta = 0, mu = 1/2 and the working
 * statistics give c~ = X~^T (y - 1/2) / n; the penalty's own zero test. */
double oracle_logistic_lambda_max(const void *X, int32_t x_is_f64, int64_t n, int64_t ldx, int32_t p,
                                  const double *y, const oracle_penalty *pen, const int32_t *groups,
                                  int32_t ngroups, const double *w, const double *cg)
{
    double *s = (double *)calloc((size_t)p, sizeof(double));
    double *c = (double *)calloc((size_t)p, sizeof(double));
    for (int64_t i = 0; i < n; ++i)
        for (int32_t j = 0; j < p; ++j) {
            double v = x_at(X, x_is_f64, ldx, i, j);
            s[j] += v * v;
        }
    for (int32_t j = 0; j < p; ++j) s[j] = s[j] > 0.0 ? sqrt(s[j] / (double)n) : 1.0;
    for (int64_t i = 0; i < n; ++i)
        for (int32_t j = 0; j < p; ++j) c[j] += (x_at(X, x_is_f64, ldx, i, j) / s[j]) * (y[i] - 0.5);
    for (int32_t j = 0; j < p; ++j) c[j] /= (double)n;
    double lm = oracle_lambda_max(p, c, pen, groups, ngroups, w, cg);
    free(s);
    free(c);
    return lm;
}
