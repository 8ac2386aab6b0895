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
                                                           const int *__restrict__ order, int chain)
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
    const auto G_g = gmem(P.G);
    const auto lambda_g = gmem(P.lambda);
    const auto beta_g = gmem(P.beta);
    const auto beta_std_g = gmem(P.beta_std);
    const auto kkt_g = gmem(P.kkt);
    const auto obj_g = gmem(P.obj);
    const auto iters_g = gmem(P.iters);
    const auto c_g = gmem(P.c);
    const auto s_g = gmem(P.s);
    const auto w_g = gmem(P.w);
    const auto gstart_g = gmem(P.gstart);
    const auto gidx_g = gmem(P.gidx);
    const auto cg_g = gmem(P.cg);
    const int p = P.p;
    const int t = threadIdx.x;
    const int lane = t % kWave, wave = t / kWave;
    // a chained launch continues from the hand-over of the kernel before it
    const int l0 = chain ? *P.lstart : 0;
    if (l0 >= P.L) return;
    const auto bws = gmem(P.bws);

    double Gr[R][CPW];
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
        for (int c = 0; c < CPW; ++c) {
            const int i = lane + 64 * r, j = NW * c + wave;
            Gr[r][c] = (i < p && j < p) ? G_g[(size_t)i * p + j] : 0.0;
        }
    for (int e = t; e < NW * CPW; e += NT) beta_s[e] = (l0 > 0 && e < p) ? bws[e] : 0.0;

    const bool mine = t < p;
    const double ct = mine ? c_g[t] : 0.0;
    const double st = mine ? s_g[t] : 1.0;
    const double wt = (mine && w_g) ? w_g[t] : 1.0;
    const double d = *P.d;
    const double yyn = *P.yyn;
    const bool grp = (P.kind == OEM_GRP_LASSO);
    if (grp) {
        for (int e = t; e <= P.ngroups; e += NT) gstart_s[e] = gstart_g[e];
        for (int e = t; e < p; e += NT) gidx_s[e] = gidx_g[e];
        for (int e = t; e < P.ngroups; e += NT) cg_s[e] = cg_g[e];
    }
    double bt = (l0 > 0 && mine) ? bws[t] : 0.0;
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

    for (int l = l0; l < P.L; ++l) {
        const double lam = lambda_g[l];
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
            if (kkt_g) kkt_g[l] = kv;
            if (obj_g) obj_g[l] = 0.5 * quad - lin + 0.5 * yyn + penv;
            if (iters_g) iters_g[l] = conv ? it : -it;
        }
        if (mine) {
            beta_g[(size_t)l * p + t] = bt / st;
            if (beta_std_g) beta_std_g[(size_t)l * p + t] = bt;
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Separable penalties (lasso, elastic net, MCP, SCAD) for p <= 128: one
// barrier per OEM update.
//
// NW waves; wave w owns the column block B_w = [CB w, CB (w + 1)) and lane l
// holds G[l + 64 r][CB w + c] (r < R, c < CB).  Wave w also owns the
// coordinates of B_w: lane l < CB keeps beta_{CB w + l} in a register.  One
// update:
//   1. every wave reads the NW partial sums of (G beta)_i for its own rows
//      (written before the last barrier), forms u_i and the new beta_i;
//   2. it broadcasts its new beta block lane by lane (readlane) and forms its
//      partial sums of G beta for all rows, the next update's input;
//   3. it writes those partials and its max |delta beta|, max |beta| into the
//      other half of a double buffer, and the workgroup meets at one barrier;
//   4. every wave reads the NW per-wave maxima and applies the stopping
//      rule, all waves taking the same decision.
// The FP64 vector rate bounds step 2 (R CB fused multiply-adds and 2 CB lane
// reads per wave); fewer waves shorten the barrier, so p <= 32 runs on one
// wave, p <= 64 on two and p <= 128 on four.
// After the stopping rule holds, the partials already hold G beta for the
// accepted beta, which gives the stationarity check and the objective.
template <int NW, int R, int CB>
__global__ __launch_bounds__(64 * NW) void path_blk_kernel(const PathDesc *__restrict__ descs,
                                                           const int *__restrict__ order, int chain)
{
    static_assert(NW * CB <= 64 * R, "each owned coordinate must be a row held by the lanes");
    __shared__ double part[2][NW][64 * R];
    __shared__ double dm[2][NW][2];
    __shared__ double fin[4][NW];

    const PathDesc P = descs[order[blockIdx.x]];
    const auto G_g = gmem(P.G);
    const auto lambda_g = gmem(P.lambda);
    const auto beta_g = gmem(P.beta);
    const auto beta_std_g = gmem(P.beta_std);
    const auto kkt_g = gmem(P.kkt);
    const auto obj_g = gmem(P.obj);
    const auto iters_g = gmem(P.iters);
    const auto c_g = gmem(P.c);
    const auto s_g = gmem(P.s);
    const auto w_g = gmem(P.w);
    const int p = P.p;
    const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
    // a chained launch continues from the hand-over of the kernel before it
    const int l0 = chain ? *P.lstart : 0;
    if (l0 >= P.L) return;

    double Gr[R][CB];
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
        for (int c = 0; c < CB; ++c) {
            const int i = lane + 64 * r, j = CB * wave + c;
            Gr[r][c] = (i < p && j < p) ? G_g[(size_t)i * p + j] : 0.0;
        }

    const int row = CB * wave + lane;              // coordinate owned by this lane
    const bool mine = (lane < CB) && (row < p);
    const double ct = mine ? c_g[row] : 0.0;
    const double st = mine ? s_g[row] : 1.0;
    const double wt = (mine && w_g) ? w_g[row] : 1.0;
    const double d = *P.d;
    const double yyn = *P.yyn;
    double bt = (l0 > 0 && mine) ? P.bws[row] : 0.0;

    // partial sums of G beta over this wave's columns, into part[buf]; NA
    // interleaved accumulators per row keep the FP64 add chains short
    auto symv = [&](int buf) {
        constexpr int NA = CB < 8 ? CB : 8;
        double acc[R][NA];
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
            for (int a = 0; a < NA; ++a) acc[r][a] = 0.0;
        const int blo = __double2loint(bt), bhi = __double2hiint(bt);
#pragma unroll
        for (int c = 0; c < CB; ++c) {
            const double bj = __hiloint2double(__builtin_amdgcn_readlane(bhi, c),
                                               __builtin_amdgcn_readlane(blo, c));
#pragma unroll
            for (int r = 0; r < R; ++r) acc[r][c % NA] += Gr[r][c] * bj;
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
#pragma unroll
            for (int h = NA / 2; h > 0; h /= 2)
#pragma unroll
                for (int a = 0; a < h; ++a) acc[r][a] += acc[r][a + h];
            part[buf][wave][lane + 64 * r] = acc[r][0];
        }
    };
    // (G beta)_row from the NW partials, summed pairwise
    auto gsum = [&](int buf) -> double {
        if (lane >= CB) return 0.0;
        double v[NW];
#pragma unroll
        for (int w = 0; w < NW; ++w) v[w] = part[buf][w][row];
#pragma unroll
        for (int h = NW / 2; h > 0; h /= 2)
#pragma unroll
            for (int w = 0; w < h; ++w) v[w] += v[w + h];
        return v[0];
    };

    int cur = 0;
    symv(cur);
    __syncthreads();

    for (int l = l0; l < P.L; ++l) {
        const double lam = lambda_g[l];
        const double lw = wt * lam;
        const Upd q = make_upd(P.kind, lw, d, P.alpha, P.gamma);
        int it = 0;
        bool conv = false;
        do {
            const double gb = gsum(cur);
            const double u = ct + (d * bt - gb);
            double dl = 0.0, mx = 0.0;
            if (mine) {
                const double bn = update_fast(P.kind, u, q, P.gamma);
                dl = fabs(bn - bt);
                mx = fabs(bn);
                bt = bn;
            }
            ++it;
            dl = lanes_max<CB>(dl);
            mx = lanes_max<CB>(mx);
            const int nxt = cur ^ 1;
            symv(nxt);
            if (lane == 0) {
                dm[nxt][wave][0] = dl;
                dm[nxt][wave][1] = mx;
            }
            __syncthreads();
            cur = nxt;
            double DL[NW], MX[NW];
#pragma unroll
            for (int w = 0; w < NW; ++w) {
                DL[w] = dm[cur][w][0];
                MX[w] = dm[cur][w][1];
            }
#pragma unroll
            for (int h = NW / 2; h > 0; h /= 2)
#pragma unroll
                for (int w = 0; w < h; ++w) {
                    DL[w] = nmax(DL[w], DL[w + h]);
                    MX[w] = nmax(MX[w], MX[w + h]);
                }
            conv = DL[0] <= P.tol * MX[0];
        } while (!conv && it < P.maxit);

        // stationarity and objective at the accepted beta (part[cur] = G beta)
        const double gbt = gsum(cur);
        double kv = 0.0, penv = 0.0, quad = 0.0, lin = 0.0;
        if (mine) {
            const double g = gbt - ct;
            if (bt == 0.0)
                kv = pos(fabs(g) - (P.kind == OEM_ENET ? P.alpha * lw : lw));
            else
                kv = fabs(g + sgn(bt) * pen_deriv(P.kind, fabs(bt), lw, P.alpha, P.gamma));
            penv = pen_value(P.kind, bt, lw, P.alpha, P.gamma);
            quad = bt * gbt;
            lin = ct * bt;
        }
        kv = wave_max(kv);
        penv = wave_sum(penv);
        quad = wave_sum(quad);
        lin = wave_sum(lin);
        if (lane == 0) {
            fin[0][wave] = kv;
            fin[1][wave] = penv;
            fin[2][wave] = quad;
            fin[3][wave] = lin;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            kv = fin[0][0];
            penv = fin[1][0];
            quad = fin[2][0];
            lin = fin[3][0];
            for (int w = 1; w < NW; ++w) {
                kv = fmax(kv, fin[0][w]);
                penv += fin[1][w];
                quad += fin[2][w];
                lin += fin[3][w];
            }
            if (kkt_g) kkt_g[l] = kv;
            if (obj_g) obj_g[l] = 0.5 * quad - lin + 0.5 * yyn + penv;
            if (iters_g) iters_g[l] = conv ? it : -it;
        }
        if (mine) {
            beta_g[(size_t)l * p + row] = bt / st;
            if (beta_std_g) beta_std_g[(size_t)l * p + row] = bt;
        }
    }
}

// Path launch plan for the register kernel: paths with p <= 64 and
// 64 < p <= 128 go to two instantiations.
int launch_paths_reg(const PathDesc *d_desc, const int *d_order, int count, int pmax, int chain,
                     hipStream_t s)
{
    if (count == 0) return OEM_OK;
    if (pmax <= 64) {
        hipLaunchKernelGGL((path_reg_kernel<4, 1, 16>), dim3(count), dim3(256), 0, s, d_desc,
                           d_order, chain);
    } else if (pmax <= 128) {
        hipLaunchKernelGGL((path_reg_kernel<8, 2, 16>), dim3(count), dim3(512), 0, s, d_desc,
                           d_order, chain);
    } else {
        return fail(OEM_E_INVAL, "register path kernel needs p <= 128");
    }
    OEM_HIP_CHECK(hipGetLastError());
    return OEM_OK;
}

#ifndef PBLK32_NW
#define PBLK32_NW 1
#endif
#ifndef PBLK64_NW
#define PBLK64_NW 2
#endif
#ifndef PBLK128_NW
#define PBLK128_NW 4
#endif
// Separable-penalty paths: p <= 32, <= 64 and <= 128 go to three
// instantiations of the block kernel (wave counts measured best at each size).
int launch_paths_blk(const PathDesc *d_desc, const int *d_order, int count, int pmax, int chain,
                     hipStream_t s)
{
    if (count == 0) return OEM_OK;
    if (pmax <= 32)
        hipLaunchKernelGGL((path_blk_kernel<PBLK32_NW, 1, 32 / PBLK32_NW>), dim3(count), dim3(64 * PBLK32_NW),
                           0, s, d_desc, d_order, chain);
    else if (pmax <= 64)
        hipLaunchKernelGGL((path_blk_kernel<PBLK64_NW, 1, 64 / PBLK64_NW>), dim3(count), dim3(64 * PBLK64_NW),
                           0, s, d_desc, d_order, chain);
    else if (pmax <= 128)
        hipLaunchKernelGGL((path_blk_kernel<PBLK128_NW, 2, 128 / PBLK128_NW>), dim3(count),
                           dim3(64 * PBLK128_NW), 0, s, d_desc, d_order, chain);
    else
        return fail(OEM_E_INVAL, "block path kernel needs p <= 128");
    OEM_HIP_CHECK(hipGetLastError());
    return OEM_OK;
}

} // namespace oem
