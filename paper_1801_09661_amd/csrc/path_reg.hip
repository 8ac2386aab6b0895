// OEM path kernel for small p: the standardised Gram lives in registers.
//
// One workgroup of NW waves runs one warm-started path (Section 2.1
// iteration, Section 2.2 updates).  Thread (wave w, lane l) holds
// G[l + 64 r][NW c + w] for r < R, c < CPW, so the p x p matrix is spread
// over the whole workgroup and never re-read from memory.  One OEM update:
//   1. each wave forms partial sums of G beta over its columns (beta
//      broadcast from LDS);
//   2. thread t < p adds the NW partials of row t in wave order, forms
//      u_t = c_t + (d beta_t - (G beta)_t) and applies the update;
//   3. max |delta beta| and max |beta| are reduced across the workgroup.
// Two barriers per update (three for group penalties).
#include "path_common.h"

namespace oem {

template <int NW, int R, int CPW>
__global__ __launch_bounds__(64 * NW) void path_reg_kernel(const PathDesc *__restrict__ descs,
                                                           const int *__restrict__ order)
{
    constexpr int NT = 64 * NW;
    constexpr int PMAX = (64 * R < NW * CPW) ? 64 * R : NW * CPW;
    __shared__ double beta_s[NW * CPW];
    __shared__ double part[NW][64 * R];
    __shared__ double u_s[PMAX];
    __shared__ double red[4][NW];
    __shared__ int gstart_s[PMAX + 1];
    __shared__ int gidx_s[PMAX];
    __shared__ double cg_s[PMAX];

    const PathDesc P = descs[order[blockIdx.x]];
    const int p = P.p;
    const int t = threadIdx.x;
    const int lane = t % kWave, wave = t / kWave;

    double Gr[R][CPW];
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
        for (int c = 0; c < CPW; ++c) {
            const int i = lane + 64 * r, j = NW * c + wave;
            Gr[r][c] = (i < p && j < p) ? P.G[(size_t)i * p + j] : 0.0;
        }
    for (int e = t; e < NW * CPW; e += NT) beta_s[e] = 0.0;

    const bool mine = t < p;
    const double ct = mine ? P.c[t] : 0.0;
    const double st = mine ? P.s[t] : 1.0;
    const double wt = (mine && P.w) ? P.w[t] : 1.0;
    const double d = *P.d;
    const double yyn = *P.yyn;
    const bool grp = (P.kind == OEM_GRP_LASSO);
    if (grp) {
        for (int e = t; e <= P.ngroups; e += NT) gstart_s[e] = P.gstart[e];
        for (int e = t; e < p; e += NT) gidx_s[e] = P.gidx[e];
        for (int e = t; e < P.ngroups; e += NT) cg_s[e] = P.cg[e];
    }
    double bt = 0.0;
    __syncthreads();

    // partial sums of (G beta) for this thread's rows; returns row t's total
    auto symv = [&]() -> double {
        double acc[R];
#pragma unroll
        for (int r = 0; r < R; ++r) acc[r] = 0.0;
#pragma unroll
        for (int c = 0; c < CPW; ++c) {
            const double bj = beta_s[NW * c + wave];
#pragma unroll
            for (int r = 0; r < R; ++r) acc[r] += Gr[r][c] * bj;
        }
#pragma unroll
        for (int r = 0; r < R; ++r) part[wave][lane + 64 * r] = acc[r];
        __syncthreads();
        double s = 0.0;
        if (mine) {
#pragma unroll
            for (int w = 0; w < NW; ++w) s += part[w][t];
        }
        return s;
    };

    auto reduce2 = [&](double &a, double &b, bool is_max_b) {
        a = wave_max(a);
        b = is_max_b ? wave_max(b) : wave_sum(b);
        if (lane == 0) {
            red[0][wave] = a;
            red[1][wave] = b;
        }
        __syncthreads();
        double ra = red[0][0], rb = red[1][0];
        for (int w = 1; w < NW; ++w) {
            ra = fmax(ra, red[0][w]);
            rb = is_max_b ? fmax(rb, red[1][w]) : rb + red[1][w];
        }
        a = ra;
        b = rb;
    };

    for (int l = 0; l < P.L; ++l) {
        const double lam = P.lambda[l];
        int it = 0;
        bool conv = false;
        while (it < P.maxit) {
            const double gb = symv();
            const double u = ct + (d * bt - gb);
            double dl = 0.0, mx = 0.0;
            if (!grp) {
                if (mine) {
                    const double bn = update1(P.kind, u, wt * lam, d, P.alpha, P.gamma);
                    dl = fabs(bn - bt);
                    mx = fabs(bn);
                    bt = bn;
                    beta_s[t] = bn;
                }
            } else {
                if (mine) u_s[t] = u;
                __syncthreads();
                for (int gi = t; gi < P.ngroups; gi += NT) {
                    const int t0 = gstart_s[gi], t1 = gstart_s[gi + 1];
                    double ss = 0.0;
                    for (int q = t0; q < t1; ++q) ss += u_s[gidx_s[q]] * u_s[gidx_s[q]];
                    const double nrm = sqrt(ss);
                    const double lam_c = cg_s[gi] * lam;
                    const double f = nrm > 0.0 ? 1.0 - lam_c / nrm : 0.0;
                    for (int q = t0; q < t1; ++q) {
                        const int j = gidx_s[q];
                        const double bn = f > 0.0 ? (u_s[j] / d) * f : 0.0;
                        dl = fmax(dl, fabs(bn - beta_s[j]));
                        mx = fmax(mx, fabs(bn));
                        beta_s[j] = bn;
                    }
                }
                __syncthreads();
                bt = mine ? beta_s[t] : 0.0;
            }
            reduce2(dl, mx, true);
            ++it;
            if (dl <= P.tol * mx) {
                conv = true;
                break;
            }
        }

        // gradient, stationarity and objective at the accepted beta
        const double gbt = symv();
        const double g = gbt - ct;
        double kv = 0.0, penv = 0.0;
        double quad = bt * gbt, lin = ct * bt;
        if (!grp) {
            if (mine) {
                const double lw = wt * lam;
                if (bt == 0.0)
                    kv = pos(fabs(g) - (P.kind == OEM_ENET ? P.alpha * lw : lw));
                else
                    kv = fabs(g + sgn(bt) * pen_deriv(P.kind, fabs(bt), lw, P.alpha, P.gamma));
                penv = pen_value(P.kind, bt, lw, P.alpha, P.gamma);
            }
        } else {
            if (mine) u_s[t] = g;
            __syncthreads();
            for (int gi = t; gi < P.ngroups; gi += NT) {
                const int t0 = gstart_s[gi], t1 = gstart_s[gi + 1];
                const double lc = lam * cg_s[gi];
                double bn = 0.0, gn = 0.0;
                for (int q = t0; q < t1; ++q) {
                    const int j = gidx_s[q];
                    bn += beta_s[j] * beta_s[j];
                    gn += u_s[j] * u_s[j];
                }
                bn = sqrt(bn);
                gn = sqrt(gn);
                double v;
                if (bn > 0.0) {
                    double ss = 0.0;
                    for (int q = t0; q < t1; ++q) {
                        const int j = gidx_s[q];
                        const double rr = u_s[j] + lc * beta_s[j] / bn;
                        ss += rr * rr;
                    }
                    v = sqrt(ss);
                } else {
                    v = pos(gn - lc);
                }
                kv = fmax(kv, v);
                penv += lc * bn;
            }
        }
        // one max and three sums across the workgroup
        kv = wave_max(kv);
        penv = wave_sum(penv);
        quad = wave_sum(quad);
        lin = wave_sum(lin);
        if (lane == 0) {
            red[0][wave] = kv;
            red[1][wave] = penv;
            red[2][wave] = quad;
            red[3][wave] = lin;
        }
        __syncthreads();
        kv = red[0][0];
        penv = red[1][0];
        quad = red[2][0];
        lin = red[3][0];
        for (int w = 1; w < NW; ++w) {
            kv = fmax(kv, red[0][w]);
            penv += red[1][w];
            quad += red[2][w];
            lin += red[3][w];
        }
        if (t == 0) {
            if (P.kkt) P.kkt[l] = kv;
            if (P.obj) P.obj[l] = 0.5 * quad - lin + 0.5 * yyn + penv;
            if (P.iters) P.iters[l] = conv ? it : -it;
        }
        if (mine) {
            P.beta[(size_t)l * p + t] = bt / st;
            if (P.beta_std) P.beta_std[(size_t)l * p + t] = bt;
        }
        __syncthreads();
    }
}

// Path launch plan for the register kernel: paths with p <= 64 and
// 64 < p <= 128 go to two instantiations.
int launch_paths_reg(const PathDesc *d_desc, const int *d_order, int count, int pmax,
                     hipStream_t s)
{
    if (count == 0) return OEM_OK;
    if (pmax <= 64) {
        hipLaunchKernelGGL((path_reg_kernel<4, 1, 16>), dim3(count), dim3(256), 0, s, d_desc,
                           d_order);
    } else if (pmax <= 128) {
        hipLaunchKernelGGL((path_reg_kernel<8, 2, 16>), dim3(count), dim3(512), 0, s, d_desc,
                           d_order);
    } else {
        return fail(OEM_E_INVAL, "register path kernel needs p <= 128");
    }
    OEM_HIP_CHECK(hipGetLastError());
    return OEM_OK;
}

} // namespace oem
