// From per-fold sums to the problems the paths solve.
//
// Problem q = 0 is the full data, q = 1 + k the training rows of fold k
// (Section 3): G_(k) = sum_{c != k} G_c, X_(k)^T y_(k) = sum_{c != k} b_c,
// summed as written (no subtraction).  Each is scaled by 1/n_q and
// standardised to unit column norms (Section 2.1): s_j = sqrt(G_jj),
// Gs = S^-1 G S^-1, cs = S^-1 c.
//
// d per problem (Section 2.1: d >= lambda_1, d = lambda_1 converges fastest,
// found by the Lanczos algorithm): FP64 Lanczos with full
// reorthogonalisation, stopped when the top Ritz pair's residual is below
// 1e-12 of the Ritz value, or the Krylov space is invariant, or it spans
// every dimension; d = theta * (1 + 1e-10).
#include <algorithm>
#include <cmath>
#include <cstdlib>

#include "path_common.h"

namespace oem {

__device__ inline void problem_rows(int q, int K, int *skip)
{
    *skip = (q == 0) ? -1 : q - 1;
}

// phase 1: per problem, the scaled diagonal gives s; c, yy/n, n_q.  With an
// intercept the problem's columns and y are centred with the means of its
// rows (from the column sums): G/n - xbar xbar^T, X^T y/n - xbar ybar,
// y^T y/n - ybar^2; the intercept itself is unpenalised and follows from
// the solution as ybar - xbar^T beta.
__global__ void combine_scale_kernel(int p, int K, int standardize, int intercept,
                                     const double *__restrict__ Gk, const double *__restrict__ bk,
                                     const double *__restrict__ yyk, const int64_t *__restrict__ nk,
                                     const double *__restrict__ csk, const double *__restrict__ ysk,
                                     double *__restrict__ cs, double *__restrict__ sc,
                                     double *__restrict__ yyn, int64_t *__restrict__ ntrain,
                                     double *__restrict__ xbar, double *__restrict__ ybar)
{
    const int q = blockIdx.y;
    int skip;
    problem_rows(q, K, &skip);
    int64_t nq = 0;
    double yy = 0.0, ys = 0.0;
    for (int c = 0; c < K; ++c) {
        if (c == skip) continue;
        nq += nk[c];
        yy += yyk[c];
        ys += ysk[c];
    }
    const double dn = (double)nq;
    const double ym = intercept ? ys / dn : 0.0;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        yyn[q] = intercept ? yy / dn - ym * ym : yy / dn;
        ybar[q] = ym;
        ntrain[q] = nq;
    }
    for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < p; j += gridDim.x * blockDim.x) {
        double gjj = 0.0, bj = 0.0, sj = 0.0;
        for (int c = 0; c < K; ++c) {
            if (c == skip) continue;
            gjj += Gk[(size_t)c * p * p + (size_t)j * p + j];
            bj += bk[(size_t)c * p + j];
            sj += csk[(size_t)c * p + j];
        }
        gjj = gjj / dn;
        double cj = bj / dn;
        const double xm = intercept ? sj / dn : 0.0;
        if (intercept) {
            gjj -= xm * xm;
            cj -= xm * ym;
        }
        xbar[(size_t)q * p + j] = xm;
        double s = 1.0;
        if (standardize) s = gjj > 0.0 ? sqrt(gjj) : 1.0;
        sc[(size_t)q * p + j] = s;
        cs[(size_t)q * p + j] = cj / s;
    }
}

// phase 2: Gs = (G / n) / (s_i s_j)
__global__ void combine_gram_kernel(int p, int K, int intercept, const double *__restrict__ Gk,
                                    const int64_t *__restrict__ ntrain, const double *__restrict__ xbar,
                                    const double *__restrict__ sc, double *__restrict__ Gs)
{
    const int q = blockIdx.y;
    int skip;
    problem_rows(q, K, &skip);
    const double dn = (double)ntrain[q];
    const size_t pp = (size_t)p * p;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < pp;
         e += (size_t)gridDim.x * blockDim.x) {
        const int i = (int)(e / p), j = (int)(e % p);
        double v = 0.0;
        for (int c = 0; c < K; ++c) {
            if (c == skip) continue;
            v += Gk[(size_t)c * pp + e];
        }
        v = v / dn;
        if (intercept) v -= xbar[(size_t)q * p + i] * xbar[(size_t)q * p + j];
        const double r = v / (sc[(size_t)q * p + i] * sc[(size_t)q * p + j]);
        Gs[(size_t)q * pp + e] = r;
    }
}

int launch_combine(oem_gram_s *h, int standardize, int intercept, hipStream_t s)
{
    const int p = h->p, K = h->K, nq = (K == 1) ? 1 : K + 1;
    dim3 g1((p + 255) / 256, nq);
    hipLaunchKernelGGL(combine_scale_kernel, g1, dim3(256), 0, s, p, K, standardize, intercept,
                       h->Gk.as<double>(), h->bk.as<double>(), h->yyk.as<double>(),
                       h->nk.as<int64_t>(), h->csk.as<double>(), h->ysk.as<double>(),
                       h->cs.as<double>(), h->sc.as<double>(), h->yyn.as<double>(),
                       h->ntrain.as<int64_t>(), h->xbar.as<double>(), h->ybar.as<double>());
    OEM_HIP_CHECK(hipGetLastError());
    const size_t pp = (size_t)p * p;
    dim3 g2((unsigned)std::min<size_t>((pp + 255) / 256, 2048), nq);
    hipLaunchKernelGGL(combine_gram_kernel, g2, dim3(256), 0, s, p, K, intercept, h->Gk.as<double>(),
                       h->ntrain.as<int64_t>(), h->xbar.as<double>(), h->sc.as<double>(),
                       h->Gs.as<double>());
    OEM_HIP_CHECK(hipGetLastError());
    return OEM_OK;
}

// ---------------------------------------------------------------- Lanczos

constexpr int kLzThreads = 256;
constexpr int kLzWaves = kLzThreads / kWave;

// The problem a Lanczos workgroup works on: from a job table (batched
// launches over problems of different p) or from strided arrays (the K + 1
// problems of one handle).
__device__ inline LzJob lz_job(const LzJob *jobs, int p, int mmax, const double *Gs_all,
                               double *V_all, double *d_out, int32_t *steps_out)
{
    if (jobs) return jobs[blockIdx.x];
    const int q = blockIdx.x;
    LzJob J;
    J.G = Gs_all + (size_t)q * p * p;
    J.V = V_all ? V_all + (size_t)q * (mmax + 1) * p : nullptr;
    J.d = d_out + q;
    J.steps = steps_out ? steps_out + q : nullptr;
    J.p = p;
    J.mmax = mmax;
    return J;
}

__device__ inline double block_sum(double v, double *red)
{
    for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o);
    const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
    __syncthreads();
    if (lane == 0) red[wave] = v;
    __syncthreads();
    double t = 0.0;
    for (int w = 0; w < kLzWaves; ++w) t += red[w];
    return t;
}

// Number of eigenvalues of the symmetric tridiagonal (a, b) that are < x
// (Sturm sequence count of the LDL^T pivots).
__device__ inline int sturm_below(const double *a, const double *b, int m, double x)
{
    int cnt = 0;
    double q = 1.0;
    for (int i = 0; i < m; ++i) {
        double bb = (i > 0) ? b[i - 1] * b[i - 1] : 0.0;
        q = (a[i] - x) - (i > 0 ? bb / q : 0.0);
        if (q == 0.0) q = -1e-300;
        if (q < 0.0) ++cnt;
    }
    return cnt;
}

// Top eigenvalue of T (m x m) by multisection on one wave; returns [lo, hi].
__device__ inline void tri_top(const double *a, const double *b, int m, double *lo_out,
                               double *hi_out)
{
    const int lane = threadIdx.x % kWave;
    double lo = -INFINITY, hi = -INFINITY;
    for (int i = 0; i < m; ++i) {
        double r = fabs(i > 0 ? b[i - 1] : 0.0) + fabs(i < m - 1 ? b[i] : 0.0);
        lo = fmax(lo, a[i]);
        hi = fmax(hi, a[i] + r);
    }
    // invariant: count(< lo) <= m - 1 (top eigenvalue >= lo), count(< hi') = m for hi' > hi
    hi = hi + fabs(hi) * 1e-15 + 1e-300;
    lo = lo - fabs(lo) * 1e-15 - 1e-300;
    for (int round = 0; round < 24; ++round) {
        if (hi - lo <= 2e-16 * fmax(fabs(lo), fabs(hi))) break;
        const double x = lo + (hi - lo) * (double)(lane + 1) / (double)(kWave + 1);
        const int below = sturm_below(a, b, m, x);
        // first lane whose point is above every eigenvalue
        const uint64_t above = __ballot(below == m);
        double nlo = lo, nhi = hi;
        if (above) {
            const int f = __ffsll((long long)above) - 1;
            nhi = lo + (hi - lo) * (double)(f + 1) / (double)(kWave + 1);
            if (f > 0) nlo = lo + (hi - lo) * (double)f / (double)(kWave + 1);
        } else {
            nlo = lo + (hi - lo) * (double)kWave / (double)(kWave + 1);
        }
        lo = nlo;
        hi = nhi;
    }
    *lo_out = lo;
    *hi_out = hi;
}

// Residual of the top Ritz pair: beta_m * |last component| of the unit
// eigenvector of T, by two steps of inverse iteration with a shift just above
// the top eigenvalue (theta' I - T is then positive definite, so the
// tridiagonal solve needs no pivoting).
__device__ inline double tri_residual(const double *a, const double *b, int m, double shift,
                                      double beta_m, double *x, double *work)
{
    for (int i = 0; i < m; ++i) x[i] = 1.0;
    for (int it = 0; it < 2; ++it) {
        // solve (shift I - T) z = x ; diag: shift - a_i ; off: -b_i
        double dprev = 0.0;
        for (int i = 0; i < m; ++i) {
            double di = shift - a[i];
            double rhs = x[i];
            if (i > 0) {
                const double l = -b[i - 1] / dprev;
                di -= l * (-b[i - 1]);
                rhs -= l * work[i - 1];
            }
            work[i] = rhs;
            x[i] = di;  // store pivot
            dprev = di;
        }
        // back substitution into x (pivots currently in x)
        double znext = 0.0;
        for (int i = m - 1; i >= 0; --i) {
            const double piv = x[i];
            const double z = (work[i] - (i < m - 1 ? -b[i] * znext : 0.0)) / piv;
            work[i] = z;
            znext = z;
        }
        double nrm = 0.0;
        for (int i = 0; i < m; ++i) nrm += work[i] * work[i];
        nrm = sqrt(nrm);
        for (int i = 0; i < m; ++i) x[i] = work[i] / nrm;
    }
    return fabs(beta_m * x[m - 1]);
}

__device__ inline double start_component(int i)
{
    uint64_t z = 0x243F6A8885A308D3ULL + (uint64_t)(i + 1) * 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    z ^= z >> 31;
    return (double)(z >> 11) * (1.0 / 9007199254740992.0) + 0.5;  // in [0.5, 1.5)
}

// Leading principal minors of x I - T: p_0 = 1, p_1 = x - a_0,
// p_i = (x - a_{i-1}) p_{i-1} - b_{i-2}^2 p_{i-2}.  x lies above every
// eigenvalue of T exactly when x I - T is positive definite, i.e. when every
// minor is positive (Sylvester's criterion).  The recurrence needs no
// division (one fused multiply-add on the dependent chain per step, where
// the pivot form p_i / p_{i-1} needs a reciprocal); only signs matter, so the
// pair (p_{i-1}, p_i) is rescaled by a power of two after every block of 8
// steps.  The entries of a block are loaded while the previous block
// computes (the loop is otherwise bound by LDS latency).
constexpr int kTriBlk = 8;

__device__ inline bool tri_above_all(const double *a, const double *b, int m, double x)
{
    double p2 = 1.0, p1 = x - a[0];
    bool ok = p1 > 0.0;
    const int nb = (m - 1) / kTriBlk;   // whole blocks of steps 1 .. nb * kTriBlk
    double an[kTriBlk], bn[kTriBlk];
    if (nb > 0) {
#pragma unroll
        for (int u = 0; u < kTriBlk; ++u) {
            an[u] = a[1 + u];
            bn[u] = b[u];
        }
    }
    for (int k = 0; k < nb && ok; ++k) {
        double ac[kTriBlk], bc[kTriBlk];
#pragma unroll
        for (int u = 0; u < kTriBlk; ++u) {
            ac[u] = an[u];
            bc[u] = bn[u];
        }
        if (k + 1 < nb) {
            const int i = 1 + (k + 1) * kTriBlk;
#pragma unroll
            for (int u = 0; u < kTriBlk; ++u) {
                an[u] = a[i + u];
                bn[u] = b[i + u - 1];
            }
        }
#pragma unroll
        for (int u = 0; u < kTriBlk; ++u) {
            const double pi = fma(x - ac[u], p1, -(bc[u] * bc[u]) * p2);
            ok = ok & (pi > 0.0);
            p2 = p1;
            p1 = pi;
        }
        int e;
        p1 = frexp(p1, &e);
        p2 = ldexp(p2, -e);
    }
    for (int i = 1 + nb * kTriBlk; i < m && ok; ++i) {
        const double pi = fma(x - a[i], p1, -(b[i - 1] * b[i - 1]) * p2);
        ok = pi > 0.0;
        p2 = p1;
        p1 = pi;
    }
    return ok;
}

// Top eigenvalue of T (m x m) by multisection on one wave, given a lower
// bound `floor` of it (the previous top Ritz value: Ritz values only grow
// with m; -inf when there is none).  With a positive floor the first round
// tests floor (1 + 2^(l - 52)) in lane l, which brackets the answer within
// a factor 2 of its distance from the floor; then 64 equally spaced points
// per round until the bracket is 2e-16 relative.  Returns [lo, hi].
__device__ inline void tri_top_pd(const double *a, const double *b, int m, double floor,
                                  double *lo_out, double *hi_out)
{
    const int lane = threadIdx.x % kWave;
    double glo = -INFINITY, ghi = -INFINITY;   // largest diagonal, Gershgorin bound
    for (int i = lane; i < m; i += kWave) {
        const double r = fabs(i > 0 ? b[i - 1] : 0.0) + fabs(i < m - 1 ? b[i] : 0.0);
        glo = fmax(glo, a[i]);
        ghi = fmax(ghi, a[i] + r);
    }
    glo = wave_max(glo);
    ghi = wave_max(ghi);
    double lo = fmax(glo, floor);
    double hi = ghi + fabs(ghi) * 1e-15 + 1e-300;
    lo = lo - fabs(lo) * 1e-15 - 1e-300;
    if (floor > 0.0 && floor < INFINITY && lo > 0.0 && lo < hi) {
        const double x = fmin(hi, lo + lo * ldexp(1.0, lane - 52));
        const uint64_t above = __ballot(tri_above_all(a, b, m, x));
        if (above) {
            const int f = __ffsll((long long)above) - 1;
            const double xf = fmin(hi, lo + lo * ldexp(1.0, f - 52));
            if (f > 0) lo = lo + lo * ldexp(1.0, f - 53);
            hi = xf;
        } else {
            lo = fmin(hi, lo + lo * ldexp(1.0, 11));
        }
    }
    for (int round = 0; round < 24; ++round) {
        if (hi - lo <= 2e-16 * fmax(fabs(lo), fabs(hi))) break;
        const double x = lo + (hi - lo) * (double)(lane + 1) / (double)(kWave + 1);
        const uint64_t above = __ballot(tri_above_all(a, b, m, x));
        double nlo = lo, nhi = hi;
        if (above) {
            const int f = __ffsll((long long)above) - 1;
            nhi = lo + (hi - lo) * (double)(f + 1) / (double)(kWave + 1);
            if (f > 0) nlo = lo + (hi - lo) * (double)f / (double)(kWave + 1);
        } else {
            nlo = lo + (hi - lo) * (double)kWave / (double)(kWave + 1);
        }
        lo = nlo;
        hi = nhi;
    }
    *lo_out = lo;
    *hi_out = hi;
}

// Residual of the top Ritz pair as in tri_residual, with the pivots of
// shift I - T = L D L^T taken from its leading minors (d_i = p_i / p_{i-1},
// off the dependent chain) and reused by both inverse-iteration solves, each
// of which is then one fused multiply-add per step in each direction:
// y_i = s_i + (b_{i-1} / d_{i-1}) y_{i-1}, z_i = (y_i + b_i z_{i+1}) / d_i.
// The entries are read in blocks of 8, one block ahead.  c[i] = b_i / d_i
// and r[i] = 1 / d_i are kept; y holds the forward and then the backward
// solution.  Infinity when a minor is not positive (shift not above every
// eigenvalue).
__device__ inline double tri_residual_pd(const double *a, const double *b, int m, double shift,
                                         double beta_m, double *r, double *y)
{
    constexpr int B = kTriBlk;
    double p2 = 1.0, p1 = shift - a[0];
    if (!(p1 > 0.0)) return INFINITY;
    r[0] = 1.0 / p1;
    bool ok = true;
    {
        const int nb = (m - 1) / B;
        double an[B], bn[B];
        if (nb > 0) {
#pragma unroll
            for (int u = 0; u < B; ++u) {
                an[u] = a[1 + u];
                bn[u] = b[u];
            }
        }
        for (int k = 0; k < nb && ok; ++k) {
            const int i0 = 1 + k * B;
            double ac[B], bc[B], rr[B];
#pragma unroll
            for (int u = 0; u < B; ++u) {
                ac[u] = an[u];
                bc[u] = bn[u];
            }
            if (k + 1 < nb) {
#pragma unroll
                for (int u = 0; u < B; ++u) {
                    an[u] = a[i0 + B + u];
                    bn[u] = b[i0 + B + u - 1];
                }
            }
#pragma unroll
            for (int u = 0; u < B; ++u) {
                const double pi = fma(shift - ac[u], p1, -(bc[u] * bc[u]) * p2);
                ok = ok & (pi > 0.0);
                rr[u] = p1 / pi;
                p2 = p1;
                p1 = pi;
            }
#pragma unroll
            for (int u = 0; u < B; ++u) r[i0 + u] = rr[u];
            int e;
            p1 = frexp(p1, &e);
            p2 = ldexp(p2, -e);
        }
        for (int i = 1 + nb * B; i < m && ok; ++i) {
            const double pi = fma(shift - a[i], p1, -(b[i - 1] * b[i - 1]) * p2);
            ok = pi > 0.0;
            r[i] = p1 / pi;
            p2 = p1;
            p1 = pi;
        }
    }
    if (!ok) return INFINITY;
    // forward solve L y = s (s = all ones, or y itself times `scale`)
    auto forward = [&](bool ones, double scale) {
        double yp = ones ? 1.0 : y[0] * scale;
        y[0] = yp;
        const int nb = (m - 1) / B;
        double bn[B], rn[B], sn[B];
        auto load = [&](int i0, double (&bb)[B], double (&rv)[B], double (&sv)[B]) {
#pragma unroll
            for (int u = 0; u < B; ++u) {
                bb[u] = b[i0 + u - 1];
                rv[u] = r[i0 + u - 1];
                sv[u] = ones ? 1.0 : y[i0 + u] * scale;
            }
        };
        if (nb > 0) load(1, bn, rn, sn);
        for (int k = 0; k < nb; ++k) {
            const int i0 = 1 + k * B;
            double bc[B], rc[B], sc[B];
#pragma unroll
            for (int u = 0; u < B; ++u) {
                bc[u] = bn[u];
                rc[u] = rn[u];
                sc[u] = sn[u];
            }
            if (k + 1 < nb) load(i0 + B, bn, rn, sn);
#pragma unroll
            for (int u = 0; u < B; ++u) {
                yp = fma(bc[u] * rc[u], yp, sc[u]);
                y[i0 + u] = yp;
            }
        }
        for (int i = 1 + nb * B; i < m; ++i) {
            yp = fma(b[i - 1] * r[i - 1], yp, ones ? 1.0 : y[i] * scale);
            y[i] = yp;
        }
    };
    // backward solve D L^T z = y into y; returns ||z||^2 and z_{m-1}
    auto backward = [&](double &zlast) -> double {
        double z = r[m - 1] * y[m - 1];
        y[m - 1] = z;
        zlast = z;
        double nrm2 = z * z;
        const int nb = (m - 1) / B;   // blocks of indices m-2 down to m-1-nb*B
        double bn[B], rn[B], yn[B];
        auto load = [&](int i0, double (&bb)[B], double (&rv)[B], double (&yv)[B]) {
#pragma unroll
            for (int u = 0; u < B; ++u) {
                bb[u] = b[i0 - u];
                rv[u] = r[i0 - u];
                yv[u] = y[i0 - u];
            }
        };
        if (nb > 0) load(m - 2, bn, rn, yn);
        for (int k = 0; k < nb; ++k) {
            const int i0 = m - 2 - k * B;
            double bc[B], rc[B], yc[B];
#pragma unroll
            for (int u = 0; u < B; ++u) {
                bc[u] = bn[u];
                rc[u] = rn[u];
                yc[u] = yn[u];
            }
            if (k + 1 < nb) load(i0 - B, bn, rn, yn);
#pragma unroll
            for (int u = 0; u < B; ++u) {
                z = rc[u] * fma(bc[u], z, yc[u]);
                y[i0 - u] = z;
                nrm2 += z * z;
            }
        }
        for (int i = m - 2 - nb * B; i >= 0; --i) {
            z = r[i] * fma(b[i], z, y[i]);
            y[i] = z;
            nrm2 += z * z;
        }
        return nrm2;
    };
    double zl = 0.0;
    forward(true, 1.0);
    double nrm2 = backward(zl);
    forward(false, 1.0 / sqrt(nrm2));   // the second solve starts from z / ||z||
    nrm2 = backward(zl);
    return fabs(beta_m * zl) / sqrt(nrm2);
}

// Convergence test of the top Ritz value, run by one wave: theta from the
// multisection, then (lane 0) the residual of the top Ritz pair; stop when it
// is below 1e-12 of theta or the Krylov space is invariant.  The next test
// step is predicted from the residual's geometric decrease since the
// previous test (0.8 of the predicted distance, between 2 and max(8, m / 2)
// steps ahead; max(8, m / 4) before there is a decrease to go by).  Lane 0
// writes the shared results.
__device__ inline void lz_test(const double *al, const double *be, int m, double beta_m,
                               bool invariant, double floor, double *rd, double *y, int &m_prev,
                               double &r_prev, double *s_theta, int *s_flag, int *s_next)
{
    double lo, hi;
    tri_top_pd(al, be, m, floor, &lo, &hi);
    if (threadIdx.x % kWave == 0) {
        const double th = 0.5 * (lo + hi);
        const double shift = hi + (hi - lo) + 1e-13 * fabs(hi) + 1e-300;
        const double res = invariant ? 0.0 : tri_residual_pd(al, be, m, shift, beta_m, rd, y);
        const double target = 1e-12 * fabs(th);
        *s_theta = th;
        *s_flag = invariant || (res <= target);
        int step = max(8, m / 4);
        if (r_prev > 0.0 && res > 0.0 && res < r_prev && res < INFINITY) {
            // 0.8 of the predicted distance, at most m / 2 ahead
            const double rate = log(res / r_prev) / (double)(m - m_prev);   // < 0
            const double need = log(target / res) / rate;                   // steps still needed
            step = (int)fmin((double)max(8, m / 2), fmax(2.0, ceil(0.8 * need)));
        }
        *s_next = m + step;
        m_prev = m;
        r_prev = res;
    }
}

constexpr int kLzWideWaves = 16;
constexpr int kLzWideThreads = 64 * kLzWideWaves;

__device__ inline double wide_block_sum(double v, double *red)
{
    v = wave_sum(v);
    const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
    __syncthreads();
    if (lane == 0) red[wave] = v;
    __syncthreads();
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < kLzWideWaves; ++w) t += red[w];
    return t;
}

// Lanczos for 128 < p <= 512 R: the same recurrence, reorthogonalisation and
// stopping rule as lanczos_kernel, laid out for memory-level parallelism.
// Wave w covers rows 64 (w % 8) + lane + 512 r and one half of the columns
// (or of the basis vectors, in the reorthogonalisation); each lane keeps 8
// (4 when R = 4) row-segment loads in flight per row, with the broadcast
// operand taken by lane reads from a register that holds 64 consecutive
// entries.  The top Ritz
// value is tested at m = 8, 16, 24, 32, 40 and then every max(8, m / 4)
// steps.
template <int R>
__global__ __launch_bounds__(kLzWideThreads) void lanczos_wide_kernel(int p_all, int mmax_all,
                                                                      const double *__restrict__ Gs_all,
                                                                      double *__restrict__ V_all,
                                                                      double *__restrict__ d_out,
                                                                      int32_t *__restrict__ steps_out,
                                                                      const LzJob *__restrict__ jobs)
{
    constexpr int PR = 512 * R;
    const LzJob J = lz_job(jobs, p_all, mmax_all, Gs_all, V_all, d_out, steps_out);
    const int p = J.p, mmax = J.mmax;
    extern __shared__ double sm[];
    double *v = sm;                 // PR: current basis vector
    double *w = v + PR;             // PR
    double *part = w + PR;          // 2 PR: partial sums of the two halves
    double *coef = part + 2 * PR;   // mmax + 1
    double *al = coef + mmax + 1;   // mmax
    double *be = al + mmax;         // mmax
    double *tx = be + mmax;         // mmax
    double *tw = tx + mmax;         // mmax
    double *red = tw + mmax;        // kLzWideWaves
    __shared__ int s_flag, s_next;
    __shared__ double s_theta;

    const auto G = gmem(J.G);
    const auto V = gmem(J.V);
    const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
    const int half = wave / 8;
    int row[R];
    bool mine[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        row[r] = 64 * (wave % 8) + lane + 512 * r;
        mine[r] = row[r] < p;
    }

    // v0 = pseudo-random positive start vector, normalised
    double ss = 0.0;
    for (int i = threadIdx.x; i < PR; i += kLzWideThreads) {
        const double x = i < p ? start_component(i) : 0.0;
        w[i] = x;
        ss += x * x;
    }
    const double nrm0 = sqrt(wide_block_sum(ss, red));
    for (int i = threadIdx.x; i < PR; i += kLzWideThreads) {
        v[i] = w[i] / nrm0;
        if (i < p) V[i] = v[i];
    }
    __syncthreads();

    // out[rows] = sum over the columns c in [c0, c1) of M[c][rows] * x_c, x
    // in LDS; M row-major with row length p (M = G or the basis V)
    auto colsum = [&](auto M, const double *x, int c0, int c1, double (&out)[R]) {
        constexpr int U = R >= 4 ? 4 : 8;   // loads in flight per lane and row
        double acc[R][4];
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
            for (int a = 0; a < 4; ++a) acc[r][a] = 0.0;
        int rc[R];
#pragma unroll
        for (int r = 0; r < R; ++r) rc[r] = mine[r] ? row[r] : 0;
        for (int cb = c0; cb < c1; cb += 64) {
            const double xv = (cb + lane < c1) ? x[cb + lane] : 0.0;
            const int xlo = __double2loint(xv), xhi = __double2hiint(xv);
            const int m = min(64, c1 - cb);
            for (int e0 = 0; e0 < m; e0 += U) {
                double gv[U][R], xs[U];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int e = e0 + u;
                    const int c = min(cb + e, c1 - 1);      // past the end: x = 0
                    xs[u] = __hiloint2double(__builtin_amdgcn_readlane(xhi, e),
                                             __builtin_amdgcn_readlane(xlo, e));
#pragma unroll
                    for (int r = 0; r < R; ++r) gv[u][r] = M[(size_t)c * p + rc[r]];
                }
#pragma unroll
                for (int u = 0; u < U; ++u)
#pragma unroll
                    for (int r = 0; r < R; ++r) acc[r][u % 4] += gv[u][r] * xs[u];
            }
        }
#pragma unroll
        for (int r = 0; r < R; ++r) out[r] = (acc[r][0] + acc[r][1]) + (acc[r][2] + acc[r][3]);
    };

    double gnorm = 0.0, theta = 0.0, floor = -INFINITY;
    int m = 0, next_test = 8, m_prev = 0;
    double r_prev = 0.0;
    if (threadIdx.x == 0) s_flag = 0;
    for (int j = 0; j < mmax; ++j) {
        // w = G v_j: two column halves, summed in order
        {
            const int ch = (p + 1) / 2;
            double o[R];
            colsum(G, v, half * ch, min(p, (half + 1) * ch), o);
#pragma unroll
            for (int r = 0; r < R; ++r) part[half * PR + row[r]] = o[r];
        }
        __syncthreads();
        double pa = 0.0, pb = 0.0;
        for (int i = threadIdx.x; i < PR; i += kLzWideThreads) {
            const double x = i < p ? part[i] + part[PR + i] : 0.0;
            w[i] = x;
            pa += x * v[i];
            pb += x * x;
        }
        const double a = wide_block_sum(pa, red);
        double before = wide_block_sum(pb, red);
        if (threadIdx.x == 0) al[j] = a;
        gnorm = fmax(gnorm, fabs(a));
        // full reorthogonalisation against v_0..v_j (classical Gram-Schmidt,
        // repeated once when it removed most of w)
        for (int pass = 0; pass < 2; ++pass) {
            // coef[mm] = <v_mm, w>: wave w takes mm = w, w + 16, ...; lanes run over rows
            for (int mm0 = wave; mm0 <= j; mm0 += 2 * kLzWideWaves) {
                const int mm1 = mm0 + kLzWideWaves;
                const auto v0 = V + (size_t)mm0 * p;
                const auto v1 = V + (size_t)min(mm1, j) * p;
                double t0 = 0.0, t1 = 0.0;
                for (int i = lane; i < p; i += kWave) {
                    t0 += v0[i] * w[i];
                    t1 += v1[i] * w[i];
                }
                t0 = wave_sum(t0);
                t1 = wave_sum(t1);
                if (lane == 0) {
                    coef[mm0] = t0;
                    if (mm1 <= j) coef[mm1] = t1;
                }
            }
            __syncthreads();
            // w -= V^T coef over v_0..v_j: two halves of the basis, summed in order
            {
                const int mh = (j + 2) / 2;
                double o[R];
                colsum(V, coef, half * mh, min(j + 1, (half + 1) * mh), o);
#pragma unroll
                for (int r = 0; r < R; ++r) part[half * PR + row[r]] = o[r];
            }
            __syncthreads();
            double pc = 0.0;
            for (int i = threadIdx.x; i < PR; i += kLzWideThreads) {
                const double x = i < p ? w[i] - (part[i] + part[PR + i]) : 0.0;
                w[i] = x;
                pc += x * x;
            }
            const double after = wide_block_sum(pc, red);
            if (after > 0.5 * before) {
                before = after;
                break;   // little cancellation: one pass suffices
            }
            before = after;
        }
        const double b = sqrt(before);
        if (threadIdx.x == 0) be[j] = b;
        m = j + 1;
        const bool invariant = (b <= 1e-14 * fmax(gnorm, 1e-300)) || (m == p);
        const bool test_now = invariant || (m == next_test) || (m == mmax);
        __syncthreads();
        if (test_now) {
            if (threadIdx.x < kWave)
                lz_test(al, be, m, b, invariant, floor, tx, tw, m_prev, r_prev, &s_theta, &s_flag,
                        &s_next);
            __syncthreads();
            theta = s_theta;
            floor = theta * (1.0 - 1e-14);
            next_test = s_next;
            if (s_flag) break;
        }
        for (int i = threadIdx.x; i < PR; i += kLzWideThreads) {
            const double x = w[i] / b;
            v[i] = x;
            if (i < p) V[(size_t)(j + 1) * p + i] = x;
        }
        __syncthreads();
    }
    // not settled within mmax steps: Gershgorin bound, as in lanczos_kernel
    double dval = theta * (1.0 + 1e-10);
    const bool ok = s_flag != 0;
    if (!ok) {
        double gm = 0.0;
        for (int i = threadIdx.x; i < p; i += kLzWideThreads) {
            double rr = 0.0;
            for (int c = 0; c < p; ++c) rr += fabs(G[(size_t)c * p + i]);
            gm = fmax(gm, rr);
        }
        gm = wave_max(gm);
        __syncthreads();
        if (lane == 0) red[wave] = gm;
        __syncthreads();
        gm = red[0];
        for (int ww = 1; ww < kLzWideWaves; ++ww) gm = fmax(gm, red[ww]);
        dval = fmax(dval, gm);
    }
    if (threadIdx.x == 0) {
        *J.d = dval;
        if (J.steps) *J.steps = ok ? m : -m;
    }
}

size_t lanczos_wide_lds_bytes(int R, int mmax)
{
    return ((size_t)4 * 512 * R + 5 * (size_t)mmax + 1 + kLzWideWaves) * sizeof(double);
}

// One workgroup per problem.  V: (mmax + 1) x p workspace per problem.
// LDS: v (p), w (p), alpha/beta/coef (mmax each), tridiagonal scratch.
__global__ __launch_bounds__(kLzThreads) void lanczos_kernel(int p_all, int mmax_all,
                                                             const double *__restrict__ Gs_all,
                                                             double *__restrict__ V_all,
                                                             double *__restrict__ d_out,
                                                             int32_t *__restrict__ steps_out,
                                                             const LzJob *__restrict__ jobs)
{
    extern __shared__ double sm[];
    const LzJob J = lz_job(jobs, p_all, mmax_all, Gs_all, V_all, d_out, steps_out);
    const int p = J.p, mmax = J.mmax;
    const auto G = gmem(J.G);
    const auto V = gmem(J.V);
    double *w = sm;                 // p
    double *al = w + p;             // mmax
    double *be = al + mmax;         // mmax
    double *coef = be + mmax;       // mmax + 1
    double *tx = coef + mmax + 1;   // mmax
    double *tw = tx + mmax;         // mmax
    double *red = tw + mmax;        // kLzWaves + 4
    __shared__ int s_flag;
    __shared__ double s_theta;

    // v0 = pseudo-random positive start vector, normalised
    double ss = 0.0;
    for (int i = threadIdx.x; i < p; i += kLzThreads) {
        const double v = start_component(i);
        V[i] = v;
        ss += v * v;
    }
    double nrm = sqrt(block_sum(ss, red));
    for (int i = threadIdx.x; i < p; i += kLzThreads) V[i] /= nrm;
    __syncthreads();

    double gnorm = 0.0;
    int m = 0;
    double theta = 0.0;
    for (int j = 0; j < mmax; ++j) {
        const auto vj = V + (size_t)j * p;
        // w = G v_j (G symmetric: column reads are coalesced across threads)
        for (int i = threadIdx.x; i < p; i += kLzThreads) {
            double acc = 0.0;
            for (int c = 0; c < p; ++c) acc += G[(size_t)c * p + i] * vj[c];
            w[i] = acc;
        }
        __syncthreads();
        double part = 0.0;
        for (int i = threadIdx.x; i < p; i += kLzThreads) part += w[i] * vj[i];
        const double a = block_sum(part, red);
        if (threadIdx.x == 0) al[j] = a;
        gnorm = fmax(gnorm, fabs(a));
        // full reorthogonalisation against v_0..v_j (classical Gram-Schmidt,
        // repeated once when it removed most of w)
        double before = 0.0;
        for (int i = threadIdx.x; i < p; i += kLzThreads) before += w[i] * w[i];
        before = block_sum(before, red);
        for (int pass = 0; pass < 2; ++pass) {
            const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
            for (int mm = wave; mm <= j; mm += kLzWaves) {
                const auto vm = V + (size_t)mm * p;
                double t = 0.0;
                for (int i = lane; i < p; i += kWave) t += vm[i] * w[i];
                for (int o = kWave / 2; o > 0; o >>= 1) t += __shfl_xor(t, o);
                if (lane == 0) coef[mm] = t;
            }
            __syncthreads();
            for (int i = threadIdx.x; i < p; i += kLzThreads) {
                double t = w[i];
                for (int mm = 0; mm <= j; ++mm) t -= coef[mm] * V[(size_t)mm * p + i];
                w[i] = t;
            }
            __syncthreads();
            double after = 0.0;
            for (int i = threadIdx.x; i < p; i += kLzThreads) after += w[i] * w[i];
            after = block_sum(after, red);
            if (after > 0.5 * before) break;   // little cancellation: one pass suffices
            before = after;
        }
        double bsq = 0.0;
        for (int i = threadIdx.x; i < p; i += kLzThreads) bsq += w[i] * w[i];
        const double b = sqrt(block_sum(bsq, red));
        if (threadIdx.x == 0) be[j] = b;
        m = j + 1;
        const bool invariant = (b <= 1e-14 * fmax(gnorm, 1e-300)) || (m == p);
        // convergence test on wave 0, every 8 steps (the Ritz values only
        // grow with m, so testing less often never accepts an earlier one)
        __syncthreads();
        const bool test_now = invariant || (m % 8 == 0) || (m == mmax);
        if (!test_now) {
            const auto vn = V + (size_t)(j + 1) * p;
            for (int i = threadIdx.x; i < p; i += kLzThreads) vn[i] = w[i] / b;
            __syncthreads();
            continue;
        }
        if (threadIdx.x < kWave) {
            double lo, hi;
            tri_top(al, be, m, &lo, &hi);
            if (threadIdx.x == 0) {
                const double th = 0.5 * (lo + hi);
                const double shift = hi + (hi - lo) + 1e-13 * fabs(hi) + 1e-300;
                const double res = invariant ? 0.0 : tri_residual(al, be, m, shift, b, tx, tw);
                s_theta = th;
                s_flag = invariant || (res <= 1e-12 * fabs(th));
            }
        }
        __syncthreads();
        theta = s_theta;
        if (s_flag) break;
        const auto vn = V + (size_t)(j + 1) * p;
        for (int i = threadIdx.x; i < p; i += kLzThreads) vn[i] = w[i] / b;
        __syncthreads();
    }
    // Lanczos did not settle within mmax steps: fall back to the Gershgorin
    // bound max_i sum_j |G_ij| >= lambda_1, which keeps the iteration a
    // majorisation (slower, but never divergent).
    double dval = theta * (1.0 + 1e-10);
    if (!s_flag) {
        double gm = 0.0;
        for (int i = threadIdx.x; i < p; i += kLzThreads) {
            double r = 0.0;
            for (int c = 0; c < p; ++c) r += fabs(G[(size_t)c * p + i]);
            gm = fmax(gm, r);
        }
        for (int o = kWave / 2; o > 0; o >>= 1) gm = fmax(gm, __shfl_xor(gm, o));
        __syncthreads();
        if (threadIdx.x % kWave == 0) red[threadIdx.x / kWave] = gm;
        __syncthreads();
        gm = red[0];
        for (int w = 1; w < kLzWaves; ++w) gm = fmax(gm, red[w]);
        dval = fmax(dval, gm);
    }
    if (threadIdx.x == 0) {
        *J.d = dval;
        if (J.steps) *J.steps = s_flag ? m : -m;
    }
}

// Lanczos for p <= 128: G spread over the registers of 64 NW threads (thread
// (wave w, lane l) holds G[l + 64 r][NW c + w]), three vectors in LDS.  The
// plain three-term recurrence with the reasoning and stopping rule of
// lanczos_mb_kernel (no basis and no reorthogonalisation: a converged Ritz
// value is accurate to O(eps ||G||) whatever the loss of orthogonality), so
// a step is one product from registers and two block sums.
static __host__ __device__ inline int lanczos_small_steps(int p) { return 2 * p < 64 ? 64 : 2 * p; }

static size_t lanczos_small_lds_bytes(int NW, int R, int p)
{
    return ((size_t)3 * (p + 1) + (size_t)NW * 64 * R + 4 * (size_t)lanczos_small_steps(p) + 2 * NW + 8) *
           sizeof(double);
}

template <int NW, int R, int CPW>
__global__ __launch_bounds__(64 * NW) void lanczos_small_kernel(int p_all, const double *__restrict__ Gs_all,
                                                                double *__restrict__ d_out,
                                                                int32_t *__restrict__ steps_out,
                                                                const LzJob *__restrict__ jobs)
{
    extern __shared__ double sm[];
    const LzJob J = lz_job(jobs, p_all, 0, Gs_all, nullptr, d_out, steps_out);
    const int p = J.p, mcap = lanczos_small_steps(p);
    const auto G = gmem(J.G);
    const int t = threadIdx.x, lane = t % kWave, wave = t / kWave;
    const int ldv = p + 1;
    double *va = sm;                          // three vectors: v_prev, v, next
    double *vb = va + ldv;
    double *vc = vb + ldv;
    double *part = vc + ldv;                  // NW x 64 R
    double *al = part + NW * 64 * R;          // mcap
    double *be = al + mcap;                   // mcap
    double *tx = be + mcap;                   // mcap
    double *tw = tx + mcap;                   // mcap
    double *red = tw + mcap;                  // 2 NW
    __shared__ int s_flag, s_next;
    __shared__ double s_theta;

    double Gr[R][CPW];
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
        for (int c = 0; c < CPW; ++c) {
            const int i = lane + 64 * r, j = NW * c + wave;
            Gr[r][c] = (i < p && j < p) ? G[(size_t)i * p + j] : 0.0;
        }
    const bool mine = t < p;
    if (t == 0) s_flag = 0;

    auto bsum = [&](double v) -> double {
        v = wave_sum(v);
        __syncthreads();
        if (lane == 0) red[wave] = v;
        __syncthreads();
        double a = 0.0;
        for (int w = 0; w < NW; ++w) a += red[w];
        return a;
    };

    double *vprev = va, *v = vb, *vn = vc;
    const double v0 = mine ? start_component(t) : 0.0;
    const double nrm0 = sqrt(bsum(v0 * v0));
    if (mine) {
        v[t] = v0 / nrm0;
        vprev[t] = 0.0;
    }
    __syncthreads();

    double gnorm = 0.0, theta = 0.0, floor = -INFINITY, beta_prev = 0.0;
    int next_test = 8, m_prev = 0, m = 0;
    double r_prev = 0.0;
    bool nonfinite = false;
    for (int j = 0; j < mcap; ++j) {
        // w = G v
        double acc[R];
#pragma unroll
        for (int r = 0; r < R; ++r) acc[r] = 0.0;
#pragma unroll
        for (int c = 0; c < CPW; ++c) {
            const int col = NW * c + wave;
            const double vcl = col < p ? v[col] : 0.0;
#pragma unroll
            for (int r = 0; r < R; ++r) acc[r] += Gr[r][c] * vcl;
        }
#pragma unroll
        for (int r = 0; r < R; ++r) part[wave * 64 * R + lane + 64 * r] = acc[r];
        __syncthreads();
        double wt = 0.0;
        if (mine)
            for (int w = 0; w < NW; ++w) wt += part[w * 64 * R + t];
        const double alpha = bsum(mine ? wt * v[t] : 0.0);
        const double rt = mine ? (wt - alpha * v[t]) - beta_prev * vprev[t] : 0.0;
        const double beta = sqrt(bsum(rt * rt));
        if (t == 0) {
            al[j] = alpha;
            be[j] = beta;
        }
        gnorm = fmax(gnorm, fabs(alpha));
        m = j + 1;
        // non-finite statistics: no bound exists (d becomes NaN, which the
        // caller reports); every thread holds the same alpha and beta
        if (!isfinite(alpha) || !isfinite(beta)) {
            nonfinite = true;
            break;
        }
        const bool invariant = beta <= 1e-14 * fmax(gnorm, 1e-300);
        const bool test_now = invariant || (m == next_test) || (m == mcap);
        if (test_now) {
            __syncthreads();
            if (t < kWave)
                lz_test(al, be, m, beta, invariant, floor, tx, tw, m_prev, r_prev, &s_theta, &s_flag,
                        &s_next);
            __syncthreads();
            theta = s_theta;
            floor = theta * (1.0 - 1e-14);
            next_test = s_next;
            if (s_flag) break;
        }
        // v_prev <- v, v <- r / beta (buffers rotate)
        if (mine) vn[t] = rt / beta;
        double *tmp = vprev;
        vprev = v;
        v = vn;
        vn = tmp;
        beta_prev = beta;
        __syncthreads();
    }
    // not settled within the step limit: Gershgorin bound, as in the other kernels
    double dval = theta * (1.0 + 1e-10);
    const bool settled = s_flag && !nonfinite;
    if (nonfinite) {
        dval = NAN;
    } else if (!settled) {
        double gm = 0.0;
        if (mine)
            for (int c = 0; c < p; ++c) gm += fabs(G[(size_t)c * p + t]);
        gm = wave_max(gm);
        __syncthreads();
        if (lane == 0) red[wave] = gm;
        __syncthreads();
        gm = red[0];
        for (int w = 1; w < NW; ++w) gm = fmax(gm, red[w]);
        dval = fmax(dval, gm);
    }
    if (t == 0) {
        *J.d = dval;
        if (J.steps) *J.steps = settled ? m : -m;
    }
}

// Lanczos kernel class of a problem size: 0, 1 register kernels (p <= 64,
// <= 128), 2..4 wide kernels (p <= 512, 1024, 2048), 5 general kernel.
static int lz_class(int p)
{
    if (p <= 64) return 0;
    if (p <= 128) return 1;
    if (p <= 512) return 2;
    if (p <= 1024) return 3;
    if (p <= 2048) return 4;
    return 5;
}

int lanczos_mmax(int p) { return p <= 128 ? p : std::min(p, 1024); }



// One launch of `count` problems of one class: strided arrays (jobs == NULL)
// or rows of a job table; pmax bounds the p of every problem in the launch.
static int launch_lz_class(int cls, int count, int pmax, int p_all, const double *Gs_all,
                           double *V_all, double *d_out, int32_t *steps_out, const LzJob *jobs,
                           hipStream_t s)
{
    if (count == 0) return OEM_OK;
    const int mmax = lanczos_mmax(pmax);
    const int p_arg = p_all, m_arg = lanczos_mmax(p_all);
    const void *kern = nullptr;
    int threads = 0;
    size_t lds = 0;
    if (cls <= 1) {
        const int NW = cls == 0 ? 4 : 8, R = cls == 0 ? 1 : 2;
        lds = lanczos_small_lds_bytes(NW, R, pmax);
        kern = cls == 0 ? (const void *)lanczos_small_kernel<4, 1, 16> : (const void *)lanczos_small_kernel<8, 2, 16>;
        threads = 64 * NW;
        OEM_HIP_CHECK(hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
        void *args[] = {(void *)&p_arg, (void *)&Gs_all, (void *)&d_out, (void *)&steps_out, (void *)&jobs};
        OEM_HIP_CHECK(hipLaunchKernel(kern, dim3(count), dim3(threads), args, lds, s));
        return OEM_OK;
    }
    if (cls <= 4) {
        const int R = cls == 2 ? 1 : (cls == 3 ? 2 : 4);
        kern = R == 1 ? (const void *)lanczos_wide_kernel<1>
             : R == 2 ? (const void *)lanczos_wide_kernel<2> : (const void *)lanczos_wide_kernel<4>;
        lds = lanczos_wide_lds_bytes(R, mmax);
        threads = kLzWideThreads;
    } else {
        kern = (const void *)lanczos_kernel;
        lds = (size_t)(pmax + 5 * mmax + 1 + kLzWaves + 4) * sizeof(double);
        threads = kLzThreads;
    }
    OEM_HIP_CHECK(hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    void *args[] = {(void *)&p_arg, (void *)&m_arg, (void *)&Gs_all, (void *)&V_all, (void *)&d_out,
                    (void *)&steps_out, (void *)&jobs};
    OEM_HIP_CHECK(hipLaunchKernel(kern, dim3(count), dim3(threads), args, lds, s));
    return OEM_OK;
}

// ------------------------------------------------------------ multi-workgroup Lanczos
// For large p (above kMbMinP) one workgroup per problem is held to one CU's
// share of L2 bandwidth while G alone is several MB per step.  This kernel
// spreads one problem over B = ceil(p / 64) workgroups: workgroup b owns
// rows [64 b, 64 b + 64) of w = G v (lane l of each wave holds row 64 b + l;
// the four waves split the columns).  For p <= 4 CPL those rows of G stay in
// registers for the whole run; larger p reads them from memory every step.
//
// The recurrence is the plain three-term Lanczos recurrence, with no
// reorthogonalisation: in floating point a Ritz value that has converged
// approximates an eigenvalue of G to O(eps ||G||) (Paige 1976); loss of
// orthogonality only adds copies of converged values, and the largest Ritz
// value still increases monotonically towards lambda_1.  A step needs one
// exchange between the workgroups: each writes its rows of w, and after one
// barrier every workgroup reads the whole w and forms alpha = v^T w,
// r = w - alpha v - beta_prev v_prev, beta = ||r|| and the next vector over all
// p rows itself.  The sums run over the same data in the same order in every
// workgroup, so all of them take identical alpha, beta and stopping
// decisions without a second exchange.  The top Ritz value is tested on the
// schedule of the single-workgroup kernels, with the same stopping rule
// (residual of the top Ritz pair below 1e-12 of its value, or an invariant
// subspace) and the Gershgorin fallback.
//
// The barrier is an arrival counter per problem with a bounded wait (a wait
// that runs out makes d NaN): each wave waits for its own stores, thread 0
// releases, arrives, polls with relaxed loads and acquires once.  It needs
// every workgroup of the launch resident at once: the launcher sizes each
// launch from the occupancy of the GPU, splitting a table of many problems
// into several launches.
constexpr int kMbRows = 64;
constexpr int kMbWaves = 4;
constexpr int kMbThreads = 64 * kMbWaves;
constexpr int kMbMinP = 128;
constexpr unsigned kMbSpinMax = 1u << 22;   // about a second of waiting per barrier

static __host__ __device__ inline int lanczos_mb_blocks(int p) { return (p + kMbRows - 1) / kMbRows; }

// Step limit of the plain recurrence: room for ghost copies past p.
static __host__ __device__ inline int lanczos_mb_steps(int p) { return p < 128 ? 256 : (2 * p < 2048 ? 2 * p : 2048); }

// per problem, after its (mmax + 1) p basis area: the two exchange buffers
// of w (2 p), the Gershgorin partials (B), then two 32-bit counters in one
// more double
static __host__ __device__ inline size_t lanczos_mb_scratch_doubles(int p)
{
    return 2 * (size_t)p + lanczos_mb_blocks(p) + 1;
}

// vectors are padded with zeros to 4 ceil(p / 4) entries (whole column shares)
static __host__ __device__ inline int lanczos_mb_pad(int p) { return 4 * ((p + kMbWaves - 1) / kMbWaves); }

static size_t lanczos_mb_lds_bytes(int p, int mcap)
{
    return (3 * (size_t)lanczos_mb_pad(p) + 4 * (size_t)mcap + kMbWaves * 64 + 64) * sizeof(double);
}

// zero the barrier counters of every problem of a launch
__global__ void lanczos_mb_reset_kernel(int count, const LzJob *__restrict__ jobs)
{
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= count) return;
    const LzJob J = jobs[q];
    double *scr = J.V + (size_t)(J.mmax + 1) * J.p;
    unsigned *ctr = reinterpret_cast<unsigned *>(scr + lanczos_mb_scratch_doubles(J.p) - 1);
    ctr[0] = 0u;
    ctr[1] = 0u;
}

// CPL > 0: each lane keeps CPL columns of its row of G in registers (p <= 4 CPL)
template <int CPL>
__global__ __launch_bounds__(kMbThreads) void lanczos_mb_kernel(int B, const LzJob *__restrict__ jobs)
{
    const int q = blockIdx.x / B, b = blockIdx.x % B;
    const LzJob J = jobs[q];
    const int p = J.p, mmax = J.mmax;
    const int Bq = lanczos_mb_blocks(p);
    if (b >= Bq) return;   // a smaller problem of the launch: not part of its barriers
    const int mcap = lanczos_mb_steps(p);
    const auto G = gmem(J.G);
    double *scr = J.V + (size_t)(mmax + 1) * p;
    const auto Wb = gmem(scr);                    // [2][p]: w of the last two steps
    const auto P2 = gmem(scr + 2 * (size_t)p);    // [Bq]: Gershgorin partials
    unsigned *ctr = reinterpret_cast<unsigned *>(scr + lanczos_mb_scratch_doubles(p) - 1);

    extern __shared__ double sm[];
    const int pv = lanczos_mb_pad(p);
    double *va = sm;                // three vectors (pv, zero past p): v_prev, v, and w / r
    double *vb = va + pv;
    double *vc = vb + pv;
    double *al = vc + pv;           // mcap
    double *be = al + mcap;         // mcap
    double *tx = be + mcap;         // mcap
    double *tw = tx + mcap;         // mcap
    double *part = tw + mcap;       // [kMbWaves][64]
    double *red = part + kMbWaves * 64;   // 64
    __shared__ int s_flag, s_fail, s_next;
    __shared__ double s_theta;

    const int t = threadIdx.x, lane = t % kWave, wave = t / kWave;
    const int row = b * kMbRows + lane;
    const bool mine = row < p;
    const int rc = mine ? row : p - 1;
    if (t == 0) {
        s_flag = 0;
        s_fail = 0;
    }
    const int cq = (p + kMbWaves - 1) / kMbWaves;
    const int c0 = wave * cq, c1 = min(p, c0 + cq);
    double g[CPL > 0 ? CPL : 1];
    if constexpr (CPL > 0) {
#pragma unroll
        for (int k = 0; k < CPL; ++k) g[k] = (c0 + k < c1) ? G[(size_t)(c0 + k) * p + rc] : 0.0;
    }

    unsigned nbar = 0;
    auto gbar = [&]() {
        ++nbar;
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        __syncthreads();
        if (t == 0 && !s_fail) {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            __hip_atomic_fetch_add(ctr, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const unsigned target = nbar * (unsigned)Bq;
            unsigned spins = 0;
            // relaxed loads while waiting (an acquire per poll would invalidate
            // the caches every time); one acquire fence after the wait
            while (__hip_atomic_load(ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
                __builtin_amdgcn_s_sleep(8);
                if (++spins > kMbSpinMax) {
                    s_fail = 1;
                    atomicOr(ctr + 1, 1u);
                    break;
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        }
        __syncthreads();
    };
    // sum over the workgroup in a fixed order (the same in every workgroup)
    auto bsum = [&](double x) -> double {
        x = wave_sum(x);
        __syncthreads();
        if (lane == 0) red[wave] = x;
        __syncthreads();
        return (red[0] + red[1]) + (red[2] + red[3]);
    };

    double *vprev = va, *v = vb, *w = vc;
    // v0: the start vector of the single-workgroup kernels, normalised
    double ss = 0.0;
    for (int i = t; i < pv; i += kMbThreads) {
        const double x = i < p ? start_component(i) : 0.0;
        v[i] = x;
        vprev[i] = 0.0;
        w[i] = 0.0;
        ss += x * x;
    }
    const double nrm0 = sqrt(bsum(ss));
    for (int i = t; i < p; i += kMbThreads) v[i] = v[i] / nrm0;
    __syncthreads();

    double gnorm = 0.0, theta = 0.0, floor = -INFINITY, beta_prev = 0.0;
    int m = 0, next_test = 8, m_prev = 0;
    double r_prev = 0.0;
    bool nonfinite = false;
    for (int j = 0; j < mcap; ++j) {
        // this workgroup's rows of w = G v
        {
            double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
            if constexpr (CPL > 0) {
                // lane l holds v[c0 + 64 h + l]; each entry reaches the whole
                // wave by readlane (no LDS traffic).  g and these registers
                // are zero past the wave's cq columns.
                double vr[CPL / 64];
#pragma unroll
                for (int h = 0; h < CPL / 64; ++h) vr[h] = (64 * h + lane < cq) ? v[c0 + 64 * h + lane] : 0.0;
#pragma unroll
                for (int k = 0; k < CPL; k += 4) {
                    a0 += g[k] * readlane_d(vr[k / 64], k % 64);
                    a1 += g[k + 1] * readlane_d(vr[k / 64], (k + 1) % 64);
                    a2 += g[k + 2] * readlane_d(vr[k / 64], (k + 2) % 64);
                    a3 += g[k + 3] * readlane_d(vr[k / 64], (k + 3) % 64);
                    // keep the scheduler from hoisting every readlane (their
                    // scalar results would not fit in the scalar registers)
                    if (k % 8 == 4) __builtin_amdgcn_sched_barrier(0);
                }
            } else {
                int c = c0;
                for (; c + 8 <= c1; c += 8) {
                    double gg[8];
#pragma unroll
                    for (int u = 0; u < 8; ++u) gg[u] = G[(size_t)(c + u) * p + rc];
                    a0 += gg[0] * v[c] + gg[4] * v[c + 4];
                    a1 += gg[1] * v[c + 1] + gg[5] * v[c + 5];
                    a2 += gg[2] * v[c + 2] + gg[6] * v[c + 6];
                    a3 += gg[3] * v[c + 3] + gg[7] * v[c + 7];
                }
                for (; c < c1; ++c) a0 += G[(size_t)c * p + rc] * v[c];
            }
            part[wave * 64 + lane] = (a0 + a1) + (a2 + a3);
        }
        __syncthreads();
        if (wave == 0 && mine)
            Wb[(size_t)(j & 1) * p + row] = (part[lane] + part[64 + lane]) + (part[128 + lane] + part[192 + lane]);
        gbar();
        if (s_fail) break;
        // the whole w; alpha, r, beta over all rows (identical in every workgroup)
        double sa = 0.0;
        for (int i = t; i < p; i += kMbThreads) {
            const double wi = Wb[(size_t)(j & 1) * p + i];
            w[i] = wi;
            sa += v[i] * wi;
        }
        const double alpha = bsum(sa);
        double sb = 0.0;
        for (int i = t; i < p; i += kMbThreads) {
            const double r = (w[i] - alpha * v[i]) - beta_prev * vprev[i];
            w[i] = r;
            sb += r * r;
        }
        const double beta = sqrt(bsum(sb));
        gnorm = fmax(gnorm, fabs(alpha));
        if (t == 0) {
            al[j] = alpha;
            be[j] = beta;
        }
        m = j + 1;
        // non-finite statistics: no bound (d becomes NaN); every workgroup
        // takes this decision on the same values
        if (!isfinite(alpha) || !isfinite(beta)) {
            nonfinite = true;
            break;
        }
        const bool invariant = beta <= 1e-14 * fmax(gnorm, 1e-300);
        const bool test_now = invariant || (m == next_test) || (m == mcap);
        __syncthreads();
        if (test_now) {
            if (t < kWave)
                lz_test(al, be, m, beta, invariant, floor, tx, tw, m_prev, r_prev, &s_theta, &s_flag,
                        &s_next);
            __syncthreads();
            theta = s_theta;
            floor = theta * (1.0 - 1e-14);
            next_test = s_next;
            if (s_flag) break;
        }
        // next vector: v_prev <- v, v <- r / beta (buffers rotate)
        for (int i = t; i < p; i += kMbThreads) w[i] = w[i] / beta;
        double *tmp = vprev;
        vprev = v;
        v = w;
        w = tmp;
        beta_prev = beta;
        __syncthreads();
    }
    // not settled within the step limit: Gershgorin bound, as in the other kernels
    double dval = theta * (1.0 + 1e-10);
    const bool ok = s_flag != 0 && !s_fail && !nonfinite;
    if (!ok && !s_fail && !nonfinite) {
        double rs = 0.0;
        if (wave == 0 && mine)
            for (int c = 0; c < p; ++c) rs += fabs(G[(size_t)c * p + row]);
        double gm = wave == 0 ? wave_max(rs) : 0.0;
        if (t == 0) P2[b] = gm;
        gbar();
        if (!s_fail) {
            if (t < Bq) red[t] = P2[t];
            __syncthreads();
            for (int bb = 0; bb < Bq; ++bb) gm = fmax(gm, red[bb]);
            dval = fmax(dval, gm);
        }
    }
    if (s_fail || nonfinite) dval = NAN;
    if (b == 0 && t == 0) {
        *J.d = dval;
        if (J.steps) *J.steps = s_fail ? kLanczosTimedOut : (ok ? m : -m);
    }
}

size_t lanczos_workspace_doubles(int p)
{
    if (p <= 128) return 0;
    const size_t basis = (size_t)(lanczos_mmax(p) + 1) * p;
    // large p: room after the basis for the multi-workgroup kernel's scratch
    return p > kMbMinP && p <= 2048 ? basis + lanczos_mb_scratch_doubles(p) : basis;
}

thread_local bool lanczos_single_workgroup = false;

static bool lanczos_mb_enabled()
{
    static const bool on = [] {
        const char *e = getenv("OEM_LANCZOS_MB");
        return !(e && e[0] == '0');
    }();
    return on;
}

// Launch the multi-workgroup kernel over a device job table (count problems,
// largest pmax).  Returns 1 (nothing launched) when it does not apply:
// switched off (OEM_LANCZOS_MB=0, or lanczos_single_workgroup on this thread:
// launches from several streams at once could hold each other's workgroups
// off the GPU), p outside (kMbMinP, 2048], or the grid cannot be resident at
// once.  Every job's V must have lanczos_mb_scratch_doubles(p) more doubles
// after its (mmax + 1) p basis.
static int launch_lanczos_mb(const LzJob *d_jobs, int count, int pmax, hipStream_t s, int share)
{
    if (!lanczos_mb_enabled() || lanczos_single_workgroup || pmax <= kMbMinP || pmax > 2048) return 1;
    const int B = lanczos_mb_blocks(pmax);
    const size_t lds = lanczos_mb_lds_bytes(pmax, lanczos_mb_steps(pmax));
    // rows of G in registers while a lane's share of columns fits (p <= 4 CPL)
    const void *kern = pmax <= 256 ? (const void *)lanczos_mb_kernel<64>
                     : pmax <= 512 ? (const void *)lanczos_mb_kernel<128>
                                   : (const void *)lanczos_mb_kernel<0>;
    OEM_HIP_CHECK(hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    int per_cu = 0, ncu = 0, dev = 0;
    OEM_HIP_CHECK(hipGetDevice(&dev));
    OEM_HIP_CHECK(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    OEM_HIP_CHECK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, kMbThreads, lds));
    // every workgroup of a launch must be resident at once: the problems go
    // in chunks, one launch after another, of as many as 1 / share of the
    // CUs hold.  share = 2 for the calls of one handle, so that the launch
    // and work of another handle on another stream (its paths, or its own
    // d launch) fit side by side; share = 1 for a batch, whose launches
    // have the GPU to themselves
    const long fit = per_cu < 1 ? 0 : (long)per_cu * (ncu / share) / B;
    if (fit < 1) return 1;
    for (int c0 = 0; c0 < count; c0 += (int)fit) {
        const int cn = (int)std::min<long>(fit, count - c0);
        const LzJob *cj = d_jobs + c0;
        hipLaunchKernelGGL(lanczos_mb_reset_kernel, dim3((cn + 63) / 64), dim3(64), 0, s, cn, cj);
        OEM_HIP_CHECK(hipGetLastError());
        int b_arg = B;
        void *args[] = {(void *)&b_arg, (void *)&cj};
        OEM_HIP_CHECK(hipLaunchKernel(kern, dim3((unsigned)((long)cn * B)), dim3(kMbThreads), args, lds, s));
    }
    return OEM_OK;
}

int launch_lanczos(oem_gram_s *h, hipStream_t s)
{
    const int p = h->p, nq = (h->K == 1) ? 1 : h->K + 1;
    const size_t ws = lanczos_workspace_doubles(p);
    if (ws) {
        int rc = h->lanczos.ensure((size_t)nq * ws * sizeof(double) + 64);
        if (rc) return rc;
        if (p > kMbMinP && p <= 2048 && lanczos_mb_enabled() && !lanczos_single_workgroup) {
            // a small job table on the device, one job per problem
            std::vector<LzJob> jobs(nq);
            for (int q = 0; q < nq; ++q)
                jobs[q] = LzJob{h->Gs.as<double>() + (size_t)q * p * p, h->lanczos.as<double>() + (size_t)q * ws,
                                h->dq.as<double>() + q, h->lzsteps.as<int32_t>() + q, p, lanczos_mmax(p)};
            rc = h->lzjobs.ensure(nq * sizeof(LzJob));
            if (rc) return rc;
            OEM_HIP_CHECK(hipMemcpyAsync(h->lzjobs.ptr, jobs.data(), nq * sizeof(LzJob), hipMemcpyHostToDevice, s));
            OEM_HIP_CHECK(hipStreamSynchronize(s));
            rc = launch_lanczos_mb(h->lzjobs.as<LzJob>(), nq, p, s, 2);
            if (rc <= 0) return rc;   // launched, or an error
        }
    }
    return launch_lz_class(lz_class(p), nq, p, p, h->Gs.as<double>(), ws ? h->lanczos.as<double>() : nullptr,
                           h->dq.as<double>(), h->lzsteps.as<int32_t>(), nullptr, s);
}

void lanczos_job_plan(std::vector<LzJob> &jobs, std::vector<LzLaunch> &launches)
{
    std::stable_sort(jobs.begin(), jobs.end(),
                     [](const LzJob &a, const LzJob &b) { return lz_class(a.p) < lz_class(b.p); });
    launches.clear();
    for (size_t i = 0; i < jobs.size();) {
        const int c = lz_class(jobs[i].p);
        size_t j = i;
        int pmax = 0;
        while (j < jobs.size() && lz_class(jobs[j].p) == c) pmax = std::max(pmax, jobs[j++].p);
        launches.push_back(LzLaunch{c, (int)i, (int)(j - i), pmax});
        i = j;
    }
}

int launch_lanczos_jobs(const LzJob *d_jobs, const std::vector<LzLaunch> &launches, hipStream_t s)
{
    for (const LzLaunch &L : launches) {
        int rc = 1;
        // the largest class: one problem over many workgroups when every
        // problem of the launch is above the threshold
        if (L.cls >= 2 && L.cls <= 4) {
            rc = launch_lanczos_mb(d_jobs + L.first, L.count, L.pmax, s, 1);
            if (rc < 0) return rc;
        }
        if (rc == 1)
            rc = launch_lz_class(L.cls, L.count, L.pmax, 0, nullptr, nullptr, nullptr, nullptr,
                                 d_jobs + L.first, s);
        if (rc) return rc;
    }
    return OEM_OK;
}

} // namespace oem
