// Penalised logistic regression (Section 4): proximal Newton with OEM as the
// inner solver.  The model is Pr(y = 1 | x) = 1 / (1 + exp(-x^T beta)), y in
// {0, 1}, no intercept; the objective is the mean negative log-likelihood
// (1/n) sum [log(1 + exp(x_i^T beta)) - y_i x_i^T beta] plus the penalty.
//
// At the current beta a Newton step needs the gradient X^T (y - mu) / n and
// the Hessian X^T W X / n, W = diag(mu (1 - mu)) (or 1/4, the bound of
// Section 4).  In standardised coordinates (columns scaled once to unit mean
// square) the quadratic model of the weighted least-squares problem is
//     q(b) = 1/2 b^T H b - c^T b,  H = S^-1 X^T W X S^-1 / n,
//     c = H b_cur + S^-1 X^T (y - mu) / n
// (c is S^-1 X^T W z / n with the working response z written out), and its
// penalised minimiser is found by OEM updates from b_cur with d = lambda_1(H)
// (1 + 1e-10).  Passes over X per Newton step:
//   * logit pass: one wave per row, lanes across columns; eta = x^T beta,
//     the weight, the residual y - mu accumulated into per-lane column sums,
//     the log-likelihood; one read of X (HBM-bound);
//   * weighted Gram pass (exact Hessian only): the FP64 matrix-core Gram
//     kernel with row weights.
// With the Hessian bound the Gram is formed once and only the logit pass
// repeats (a majorise-minimise iteration).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "path_common.h"

namespace oem {

constexpr int kLogitThreads = 256;
constexpr int kLogitWaves = kLogitThreads / kWave;
constexpr int kLogitBlocks = 512;

__device__ inline double softplus_d(double t) { return t > 0.0 ? t + log1p(exp(-t)) : log1p(exp(t)); }

// R = columns per lane / 64 (p <= 64 R); U rows in flight per wave.
template <typename XT, int R, int U>
__global__ __launch_bounds__(kLogitThreads) void logit_pass_kernel(
    const XT *__restrict__ X, int64_t n, int64_t ldx, int p, const double *__restrict__ y,
    const double *__restrict__ bstd, const double *__restrict__ sc, int bound,
    double *__restrict__ w_out, double *__restrict__ gpart, double *__restrict__ lpart)
{
    extern __shared__ double sm[];   // reductions: kLogitWaves x p, then kLogitWaves
    const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
    double breg[R], acc[R];
#pragma unroll
    for (int c = 0; c < R; ++c) {
        const int j = lane + kWave * c;
        breg[c] = j < p ? bstd[j] / sc[j] : 0.0;
        acc[c] = 0.0;
    }
    double loss = 0.0;
    const int64_t stride = (int64_t)gridDim.x * kLogitWaves;
    for (int64_t i0 = (int64_t)blockIdx.x * kLogitWaves + wave; i0 < n; i0 += stride * U) {
        double xv[U][R];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t i = i0 + u * stride;
            const XT *row = X + (i < n ? i : i0) * ldx;
#pragma unroll
            for (int c = 0; c < R; ++c) {
                const int j = lane + kWave * c;
                xv[u][c] = (j < p && i < n) ? (double)row[j] : 0.0;
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t i = i0 + u * stride;
            double dot = 0.0;
#pragma unroll
            for (int c = 0; c < R; ++c) dot += xv[u][c] * breg[c];
            const double eta = wave_sum(dot);
            if (i < n) {
                const double mu = 1.0 / (1.0 + exp(-eta));
                const double yi = y[i];
                const double r = yi - mu;
#pragma unroll
                for (int c = 0; c < R; ++c) acc[c] += xv[u][c] * r;
                if (lane == 0) {
                    if (w_out) w_out[i] = bound ? 0.25 : mu * (1.0 - mu);
                    loss += softplus_d(eta) - yi * eta;
                }
            }
        }
    }
    // the waves' column sums and losses, combined in wave order
#pragma unroll
    for (int c = 0; c < R; ++c) {
        const int j = lane + kWave * c;
        if (j < p) sm[wave * p + j] = acc[c];
    }
    if (lane == 0) sm[kLogitWaves * p + wave] = loss;
    __syncthreads();
    for (int j = threadIdx.x; j < p; j += kLogitThreads) {
        double t = sm[j];
        for (int w = 1; w < kLogitWaves; ++w) t += sm[w * p + j];
        gpart[(size_t)blockIdx.x * p + j] = t;
    }
    if (threadIdx.x == 0) {
        double t = sm[kLogitWaves * p];
        for (int w = 1; w < kLogitWaves; ++w) t += sm[kLogitWaves * p + w];
        lpart[blockIdx.x] = t;
    }
}

// g~_j = sum_b gpart[b][j] / (n s_j) (blocks in order); loss = sum_b lpart[b] / n
__global__ void logit_finish_kernel(const double *__restrict__ gpart, const double *__restrict__ lpart,
                                    int nblk, int p, double n, const double *__restrict__ sc,
                                    double *__restrict__ gstd, double *__restrict__ loss)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j < p) {
        double t = 0.0;
        for (int b = 0; b < nblk; ++b) t += gpart[(size_t)b * p + j];
        gstd[j] = t / n / sc[j];
    }
    if (j == 0) {
        double t = 0.0;
        for (int b = 0; b < nblk; ++b) t += lpart[b];
        *loss = t / n;
    }
}

// H = scale (G / n) / (s_i s_j)
__global__ void logit_hess_kernel(const double *__restrict__ G, int p, double n, const double *__restrict__ sc,
                                  double scale, double *__restrict__ H)
{
    const size_t pp = (size_t)p * p;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < pp; e += (size_t)gridDim.x * blockDim.x) {
        const int i = (int)(e / p), j = (int)(e % p);
        H[e] = scale * (G[e] / n) / (sc[i] * sc[j]);
    }
}

// c = H b + g~ (one thread per row of H)
__global__ void logit_model_kernel(const double *__restrict__ H, int p, const double *__restrict__ b,
                                   const double *__restrict__ gstd, double *__restrict__ c)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= p) return;
    double t = 0.0;
    for (int j = 0; j < p; ++j) t += H[(size_t)i * p + j] * b[j];
    c[i] = t + gstd[i];
}

// max |bnew - bcur|, max |bnew| and d into out[0..2]; bcur <- bnew
__global__ __launch_bounds__(kLogitThreads) void logit_step_kernel(const double *__restrict__ bnew,
                                                                   double *__restrict__ bcur, int p,
                                                                   const double *__restrict__ d,
                                                                   double *__restrict__ out)
{
    __shared__ double red[2 * kLogitWaves];
    double dl = 0.0, mx = 0.0;
    for (int j = threadIdx.x; j < p; j += kLogitThreads) {
        dl = fmax(dl, fabs(bnew[j] - bcur[j]));
        mx = fmax(mx, fabs(bnew[j]));
        bcur[j] = bnew[j];
    }
    dl = wave_max(dl);
    mx = wave_max(mx);
    if (threadIdx.x % kWave == 0) {
        red[threadIdx.x / kWave] = dl;
        red[kLogitWaves + threadIdx.x / kWave] = mx;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < kLogitWaves; ++w) {
            dl = fmax(dl, red[w]);
            mx = fmax(mx, red[kLogitWaves + w]);
        }
        dl = fmax(dl, red[0]);
        mx = fmax(mx, red[kLogitWaves]);
        out[0] = dl;
        out[1] = mx;
        out[2] = *d;
    }
}

// Stationarity violation and objective of the logistic problem at b
// (standardised) from its gradient -g~: the rules of the path kernels with
// the smooth part's gradient in place of G b - c.  One workgroup.
__global__ __launch_bounds__(kLogitThreads) void logit_kkt_kernel(PathDesc P, const double *__restrict__ b,
                                                                  const double *__restrict__ gstd,
                                                                  const double *__restrict__ loss,
                                                                  double *__restrict__ kkt,
                                                                  double *__restrict__ obj)
{
    __shared__ double red[2 * kLogitWaves];
    const double lam = *P.lambda;
    const int p = P.p;
    double kv = 0.0, penv = 0.0;
    if (!group_penalty(P.kind)) {
        for (int i = threadIdx.x; i < p; i += kLogitThreads) {
            const double lw = (P.w ? P.w[i] : 1.0) * lam;
            const double g = -gstd[i], bi = b[i];
            double v;
            if (bi == 0.0) v = pos(fabs(g) - (P.kind == OEM_ENET ? P.alpha * lw : lw));
            else v = fabs(g + sgn(bi) * pen_deriv(P.kind, fabs(bi), lw, P.alpha, P.gamma));
            kv = fmax(kv, v);
            penv += pen_value(P.kind, bi, lw, P.alpha, P.gamma);
        }
    } else {
        for (int gi = threadIdx.x; gi < P.ngroups; gi += kLogitThreads) {
            const double cgk = P.cg[gi];
            const double lc = group_lam_c(P.kind, cgk, lam, P.tau);
            double bn = 0.0, gn = 0.0, l1w = 0.0;
            const int t0 = P.gstart[gi], t1 = P.gstart[gi + 1];
            for (int t = t0; t < t1; ++t) {
                const int j = P.gidx[t];
                bn += b[j] * b[j];
                gn += gstd[j] * gstd[j];
                l1w += (P.w ? P.w[j] : 1.0) * fabs(b[j]);
            }
            bn = sqrt(bn);
            gn = sqrt(gn);
            double v;
            if (P.kind == OEM_SGL) {
                double ss = 0.0;
                for (int t = t0; t < t1; ++t) {
                    const int j = P.gidx[t];
                    const double lt = lam * P.tau * (P.w ? P.w[j] : 1.0);
                    const double g = -gstd[j];
                    const double r = (bn == 0.0 || b[j] == 0.0) ? pos(fabs(g) - lt)
                                                                 : g + lc * b[j] / bn + lt * sgn(b[j]);
                    ss += r * r;
                }
                v = bn == 0.0 ? pos(sqrt(ss) - lc) : sqrt(ss);
            } else if (bn > 0.0) {
                const double dp = group_pen_deriv(P.kind, bn, lc, P.gamma);
                double ss = 0.0;
                for (int t = t0; t < t1; ++t) {
                    const int j = P.gidx[t];
                    const double r = -gstd[j] + dp * b[j] / bn;
                    ss += r * r;
                }
                v = sqrt(ss);
            } else {
                v = pos(gn - lc);
            }
            kv = fmax(kv, v);
            penv += group_pen_value(P.kind, bn, l1w, cgk, lam, P.gamma, P.tau);
        }
    }
    kv = wave_max(kv);
    penv = wave_sum(penv);
    if (threadIdx.x % kWave == 0) {
        red[threadIdx.x / kWave] = kv;
        red[kLogitWaves + threadIdx.x / kWave] = penv;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double k2 = red[0], p2 = red[kLogitWaves];
        for (int w = 1; w < kLogitWaves; ++w) {
            k2 = fmax(k2, red[w]);
            p2 += red[kLogitWaves + w];
        }
        if (kkt) *kkt = k2;
        if (obj) *obj = *loss + p2;
    }
}

// ---------------------------------------------------------------- host

template <typename XT, int R>
static int launch_logit_r(const XT *X, int64_t n, int64_t ldx, int p, const double *y, const double *bstd,
                          const double *sc, int bound, double *w_out, double *gpart, double *lpart,
                          hipStream_t s)
{
    constexpr int U = R <= 4 ? 4 : (R <= 8 ? 2 : 1);
    const size_t lds = ((size_t)kLogitWaves * p + kLogitWaves) * sizeof(double);
    const void *k = (const void *)logit_pass_kernel<XT, R, U>;
    OEM_HIP_CHECK(hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    hipLaunchKernelGGL((logit_pass_kernel<XT, R, U>), dim3(kLogitBlocks), dim3(kLogitThreads), lds, s, X, n,
                       ldx, p, y, bstd, sc, bound, w_out, gpart, lpart);
    OEM_HIP_CHECK(hipGetLastError());
    return OEM_OK;
}

template <typename XT>
static int launch_logit(const XT *X, int64_t n, int64_t ldx, int p, const double *y, const double *bstd,
                        const double *sc, int bound, double *w_out, double *gpart, double *lpart,
                        hipStream_t s)
{
    const int r = (p + kWave - 1) / kWave;
    if (r <= 1) return launch_logit_r<XT, 1>(X, n, ldx, p, y, bstd, sc, bound, w_out, gpart, lpart, s);
    if (r <= 2) return launch_logit_r<XT, 2>(X, n, ldx, p, y, bstd, sc, bound, w_out, gpart, lpart, s);
    if (r <= 4) return launch_logit_r<XT, 4>(X, n, ldx, p, y, bstd, sc, bound, w_out, gpart, lpart, s);
    if (r <= 8) return launch_logit_r<XT, 8>(X, n, ldx, p, y, bstd, sc, bound, w_out, gpart, lpart, s);
    if (r <= 16) return launch_logit_r<XT, 16>(X, n, ldx, p, y, bstd, sc, bound, w_out, gpart, lpart, s);
    return launch_logit_r<XT, 32>(X, n, ldx, p, y, bstd, sc, bound, w_out, gpart, lpart, s);
}

struct LogitRun {
    oem_gram_s *h = nullptr;
    const void *X;
    int64_t n, ldx;
    int p, xdt;
    const double *y;
    double *w, *gpart, *lpart, *gstd, *loss, *c, *bcur, *bnew, *bzero, *out;
};

static int logit_pass(LogitRun &R, const double *bstd, int bound, bool want_w, hipStream_t s)
{
    int rc;
    if (R.xdt == OEM_X_F64)
        rc = launch_logit<double>(static_cast<const double *>(R.X), R.n, R.ldx, R.p, R.y, bstd,
                                  R.h->sc.as<double>(), bound, want_w ? R.w : nullptr, R.gpart, R.lpart, s);
    else
        rc = launch_logit<float>(static_cast<const float *>(R.X), R.n, R.ldx, R.p, R.y, bstd,
                                 R.h->sc.as<double>(), bound, want_w ? R.w : nullptr, R.gpart, R.lpart, s);
    if (rc) return rc;
    hipLaunchKernelGGL(logit_finish_kernel, dim3((R.p + 255) / 256), dim3(256), 0, s, R.gpart, R.lpart,
                       kLogitBlocks, R.p, (double)R.n, R.h->sc.as<double>(), R.gstd, R.loss);
    OEM_HIP_CHECK(hipGetLastError());
    return OEM_OK;
}

// H and d: at the current point from the weighted Gram (exact Hessian), or
// 1/4 of the unweighted Gram (bound)
static int logit_hessian(LogitRun &R, int bound, hipStream_t s)
{
    oem_gram_s *h = R.h;
    const size_t pp = (size_t)R.p * R.p;
    if (!bound) {
        int rc = oem_gram_reset(h, s);
        rc = rc ? rc : launch_gram_weighted(h, R.X, R.n, R.ldx, R.y, R.w, s);
        if (rc) return rc;
    }
    const unsigned blocks = (unsigned)std::min<size_t>((pp + 255) / 256, 2048);
    hipLaunchKernelGGL(logit_hess_kernel, dim3(blocks), dim3(256), 0, s, h->Gk.as<double>(), R.p, (double)R.n,
                       h->sc.as<double>(), bound ? 0.25 : 1.0, h->Gs.as<double>());
    OEM_HIP_CHECK(hipGetLastError());
    return launch_lanczos(h, s);
}

int logistic_path(oem_gram_s *h, const void *X, int64_t n, int64_t ldx, const double *y,
                  const oem_penalty *pen, int npen, const oem_path_opts *o, const oem_logistic_opts *lo,
                  const int32_t *d_gstart, const int32_t *d_gidx, int ngroups, const double *d_w,
                  const double *d_cg, double *beta, double *lambda, int32_t *newton_iters, double *kkt,
                  double *obj, hipStream_t s)
{
    const int p = h->p;
    LogitRun R;
    R.h = h;
    R.X = X;
    R.n = n;
    R.ldx = ldx;
    R.p = p;
    R.xdt = h->xdt;
    R.y = y;
    const int L = o->nlambda;
    const size_t nl = (size_t)npen * L;
    const int bound = lo->hessian_bound ? 1 : 0;
    // workspace: w (n), block partials, p-vectors, scalars, own lambda,
    // penalties and path descriptors
    const size_t doubles = (size_t)n + (size_t)kLogitBlocks * p + kLogitBlocks + 5 * (size_t)p + 8 + nl;
    const size_t bytes = doubles * sizeof(double) + npen * sizeof(oem_penalty) + nl * sizeof(PathDesc) + 256;
    int rc = h->betaw.ensure(bytes);
    if (rc) return rc;
    double *b0 = h->betaw.as<double>();
    R.w = b0;
    R.gpart = R.w + n;
    R.lpart = R.gpart + (size_t)kLogitBlocks * p;
    R.gstd = R.lpart + kLogitBlocks;
    R.c = R.gstd + p;
    R.bcur = R.c + p;
    R.bnew = R.bcur + p;
    R.bzero = R.bnew + p;
    R.loss = R.bzero + p;
    R.out = R.loss + 1;
    double *zero1 = R.out + 3;
    double *lam = lambda ? lambda : zero1 + 4;
    oem_penalty *d_pens = reinterpret_cast<oem_penalty *>(zero1 + 4 + nl);
    char *desc_at = reinterpret_cast<char *>(d_pens + npen);
    desc_at = reinterpret_cast<char *>((reinterpret_cast<uintptr_t>(desc_at) + 15) & ~uintptr_t(15));
    PathDesc *d_desc = reinterpret_cast<PathDesc *>(desc_at);

    // column scales (unit mean square) and the unweighted Gram
    rc = oem_gram_reset(h, s);
    rc = rc ? rc : launch_gram(h, X, n, ldx, y, 0, nullptr, s);
    if (rc) return rc;
    h->rows_seen = n;
    h->derived_valid = false;
    rc = launch_combine(h, 1, 0, s);
    rc = rc ? rc : launch_fill_f64(R.bzero, (size_t)p + 8, 0.0, s);   // bzero, loss, out, zero1
    if (rc) return rc;
    // lambda grids from c~ at beta = 0 (mu = 1/2): S^-1 X^T (y - 1/2) / n
    if (o->lambda) {
        OEM_HIP_CHECK(hipMemcpyAsync(lam, o->lambda, nl * sizeof(double), hipMemcpyHostToDevice, s));
    } else {
        rc = logit_pass(R, R.bzero, 1, false, s);
        if (rc) return rc;
        OEM_HIP_CHECK(hipMemcpyAsync(d_pens, pen, npen * sizeof(oem_penalty), hipMemcpyHostToDevice, s));
        rc = launch_lambda_grid(R.gstd, p, d_gstart, d_gidx, ngroups, d_w, d_cg, d_pens, npen, L,
                                o->lambda_min_ratio, lam, s);
        if (rc) return rc;
    }
    if (bound) {
        rc = logit_hessian(R, 1, s);
        if (rc) return rc;
    }
    // one single-lambda solve per (penalty, lambda): from bcur into bnew
    std::vector<PathDesc> descs(nl);
    for (int i = 0; i < npen; ++i)
        for (int l = 0; l < L; ++l) {
            PathDesc &d = descs[(size_t)i * L + l];
            d = PathDesc{};
            d.G = h->Gs.as<double>();
            d.c = R.c;
            d.s = h->sc.as<double>();
            d.yyn = zero1;
            d.d = h->dq.as<double>();
            d.lambda = lam + (size_t)i * L + l;
            d.beta = beta + ((size_t)i * L + l) * p;
            d.beta_std = R.bnew;
            d.gstart = d_gstart;
            d.gidx = d_gidx;
            d.w = d_w;
            d.cg = d_cg;
            d.p = p;
            d.L = 1;
            d.kind = pen[i].kind;
            d.ngroups = ngroups;
            d.alpha = pen[i].alpha;
            d.gamma = pen[i].gamma;
            d.tau = pen[i].tau;
            d.tol = o->tol;
            d.maxit = o->maxit;
            d.beta_init = R.bcur;
        }
    OEM_HIP_CHECK(hipMemcpyAsync(d_desc, descs.data(), nl * sizeof(PathDesc), hipMemcpyHostToDevice, s));
    std::vector<int32_t> newton(nl, 0);
    int status = OEM_OK;
    double host_out[3];
    for (int i = 0; i < npen; ++i) {
        rc = launch_fill_f64(R.bcur, p, 0.0, s);
        if (rc) return rc;
        for (int l = 0; l < L; ++l) {
            const size_t il = (size_t)i * L + l;
            int t = 0;
            bool conv = false;
            while (t < lo->newton_maxit) {
                rc = logit_pass(R, R.bcur, bound, !bound, s);
                if (!rc && !bound) rc = logit_hessian(R, 0, s);
                if (rc) return rc;
                hipLaunchKernelGGL(logit_model_kernel, dim3((p + 255) / 256), dim3(256), 0, s, h->Gs.as<double>(),
                                   p, R.bcur, R.gstd, R.c);
                OEM_HIP_CHECK(hipGetLastError());
                rc = launch_paths_general(d_desc + il, 1, p, s);
                if (rc) return rc;
                hipLaunchKernelGGL(logit_step_kernel, dim3(1), dim3(kLogitThreads), 0, s, R.bnew, R.bcur, p,
                                   h->dq.as<double>(), R.out);
                OEM_HIP_CHECK(hipGetLastError());
                OEM_HIP_CHECK(hipMemcpyAsync(host_out, R.out, sizeof(host_out), hipMemcpyDeviceToHost, s));
                OEM_HIP_CHECK(hipStreamSynchronize(s));
                ++t;
                const double dd = host_out[2];
                if (!(std::isfinite(dd) && dd > 0.0))
                    return fail(OEM_E_INVAL, "the Hessian bound d of a Newton step is not a finite positive number");
                const int kd = pen[i].kind;
                if ((kd == OEM_MCP || kd == OEM_GRP_MCP) && !(pen[i].gamma * dd > 1.0))
                    return fail(OEM_E_INVAL, "MCP needs gamma * d > 1 at every Newton step");
                if ((kd == OEM_SCAD || kd == OEM_GRP_SCAD) && !((pen[i].gamma - 1.0) * dd > 1.0))
                    return fail(OEM_E_INVAL, "SCAD needs (gamma - 1) d > 1 at every Newton step");
                if (host_out[0] <= lo->newton_tol * host_out[1]) {
                    conv = true;
                    break;
                }
            }
            newton[il] = conv ? t : -t;
            if (!conv) status = OEM_NOT_CONVERGED;
            if (kkt || obj) {
                rc = logit_pass(R, R.bcur, bound, false, s);
                if (rc) return rc;
                hipLaunchKernelGGL(logit_kkt_kernel, dim3(1), dim3(kLogitThreads), 0, s, descs[il], R.bcur, R.gstd,
                                   R.loss, kkt ? kkt + il : nullptr, obj ? obj + il : nullptr);
                OEM_HIP_CHECK(hipGetLastError());
            }
        }
    }
    if (newton_iters)
        OEM_HIP_CHECK(hipMemcpyAsync(newton_iters, newton.data(), nl * sizeof(int32_t), hipMemcpyHostToDevice, s));
    OEM_HIP_CHECK(hipStreamSynchronize(s));
    if (status != OEM_OK) set_error("some lambda reached the Newton step limit before the coefficients settled");
    return status;
}

} // namespace oem
