// OEM path kernel for larger p (128 < p <= 2048): the Gram streams from L2.
//
// One workgroup of 8 waves runs one warm-started path (Section 2.1
// iteration, Section 2.2 updates).  Wave w, lane l owns the coordinates
// i = 64 w + l + 512 r (r < R) and keeps beta_i in registers.  Only the
// columns of G whose coefficient is nonzero enter G beta, so each update
// reads p x |active| entries of G (columns are contiguous: G is symmetric and
// row-major, so column j is row j).  One update:
//   1. every lane holds (G beta)_i for its coordinates, forms u_i and the new
//      beta_i (group lasso: u goes through LDS and a barrier first, then each
//      lane reads its group's entries for the group norm);
//   2. each wave publishes its nonzero coefficients as (index, value) pairs,
//      compacted within the wave, into its own segment of a double-buffered
//      list, with its max |delta beta| and max |beta|; one barrier;
//   3. every wave walks the eight segments as one list: lane k reads entry k
//      of a 64-entry chunk and the entries are broadcast with lane reads; for
//      each entry j the wave loads G[j][rows] (one 512-byte row segment per
//      load, many in flight) and accumulates G beta for its rows;
//   4. the eight per-wave maxima give the stopping rule, the same decision
//      in every wave.
// When the stopping rule holds, step 3 has already formed G beta for the
// accepted beta, which gives the stationarity check and the objective.
//
// One CU draws only some tens of GB/s from L2, so the columns of the active
// set are also kept in LDS: after a lambda whose support changed, the first
// nonzero coordinates (as many columns as fit) get cache slots and their
// columns are loaded once; step 3 then reads those columns from LDS and only
// the rest from L2.
#include "path_common.h"

namespace oem {

constexpr int kStreamWaves = 8;
constexpr int kStreamThreads = 64 * kStreamWaves;

struct StreamLds {
    int *lj;        // [2][NW][SEG] coefficient indices
    double *lb;     // [2][NW][SEG] coefficient values
    int *lcnt;      // [2][NW]
    double *dm;     // [2][NW][2]
    double *fin;    // [4][NW]
    double *us;     // [NW * SEG] u or gradient (group penalties)
    int *gof;       // [NW * SEG] group of each coordinate
    double *cache;  // [C][p] cached columns of G
    double *cb;     // [2][64] beta of the cached coordinates
    int *cj;        // [64] coordinate of each cache slot
    int *wcnt;      // [NW] per-wave counts (cache refill)
};

constexpr int kCacheMax = 64;            // cached columns at most (one lane-read chunk)
constexpr size_t kStreamLdsLimit = 160 * 1024;

size_t path_stream_lds_bytes(int R, int p, int cols)
{
    const size_t seg = 64 * (size_t)R, nw = kStreamWaves;
    return 2 * nw * seg * (sizeof(int) + sizeof(double)) + 2 * nw * sizeof(int) + 2 * nw * 2 * sizeof(double) +
           4 * nw * sizeof(double) + nw * seg * (sizeof(double) + sizeof(int)) +
           (size_t)cols * p * sizeof(double) + 2 * kCacheMax * sizeof(double) + kCacheMax * sizeof(int) +
           nw * sizeof(int) + 64;
}

// Columns of G that fit in LDS next to the kernel's other arrays.
int path_stream_cache_cols(int R, int pmax)
{
    const size_t base = path_stream_lds_bytes(R, pmax, 0);
    if (base >= kStreamLdsLimit) return 0;
    const size_t c = (kStreamLdsLimit - base) / ((size_t)pmax * sizeof(double));
    return (int)std::min<size_t>(c, kCacheMax);
}

template <int R>
__global__ __launch_bounds__(kStreamThreads) void path_stream_kernel(const PathDesc *__restrict__ descs,
                                                                     const int *__restrict__ order,
                                                                     int cache_cols, int chain)
{
    constexpr int NW = kStreamWaves, SEG = 64 * R;
    extern __shared__ double smem_d[];
    StreamLds S;
    S.lb = smem_d;                                          // 2 NW SEG doubles
    S.dm = S.lb + 2 * NW * SEG;                             // 4 NW
    S.fin = S.dm + 4 * NW;                                  // 4 NW
    S.us = S.fin + 4 * NW;                                  // NW SEG
    S.lj = reinterpret_cast<int *>(S.us + NW * SEG);        // 2 NW SEG
    S.lcnt = S.lj + 2 * NW * SEG;                           // 2 NW
    S.gof = S.lcnt + 2 * NW;                                // NW SEG
    S.cj = S.gof + NW * SEG;                                // kCacheMax
    S.wcnt = S.cj + kCacheMax;                              // NW
    S.cb = reinterpret_cast<double *>(S.wcnt + NW + (NW % 2));  // 2 kCacheMax (8-byte aligned)
    S.cache = S.cb + 2 * kCacheMax;                         // cache_cols x p

    const PathDesc P = descs[order[blockIdx.x]];
    const int p = P.p;
    // a chained launch continues from the hand-over of the kernel before it
    const int l0 = chain ? *P.lstart : 0;
    if (l0 >= P.L) return;
    const auto bws = gmem(P.bws);
    const auto Gg = gmem(P.G);
    const auto gstart = gmem(P.gstart);
    const auto gidx = gmem(P.gidx);
    const auto cgw = gmem(P.cg);
    const auto lambda_g = gmem(P.lambda);
    const auto beta_g = gmem(P.beta);
    const auto beta_std_g = gmem(P.beta_std);
    const auto kkt_g = gmem(P.kkt);
    const auto obj_g = gmem(P.obj);
    const auto iters_g = gmem(P.iters);
    const auto c_g = gmem(P.c);
    const auto s_g = gmem(P.s);
    const auto w_g = gmem(P.w);
    const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
    const bool grp = (P.kind == OEM_GRP_LASSO);
    const double d = *P.d;
    const double yyn = *P.yyn;
    const double inv_d = 1.0 / d;

    int row[R];
    bool mine[R];
    double ct[R], st[R], wt[R], bt[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        row[r] = 64 * wave + lane + 512 * r;
        mine[r] = row[r] < p;
        ct[r] = mine[r] ? c_g[row[r]] : 0.0;
        st[r] = mine[r] ? s_g[row[r]] : 1.0;
        wt[r] = (mine[r] && w_g) ? w_g[row[r]] : 1.0;
        bt[r] = (l0 > 0 && mine[r]) ? bws[row[r]] : 0.0;
    }
    int myslot[R];        // cache slot of this lane's coordinate, -1 if not cached
#pragma unroll
    for (int r = 0; r < R; ++r) myslot[r] = -1;
    int ncached = 0;      // slots in use (uniform)
    // some coordinate of this lane changed between zero and nonzero (a warm
    // start counts as a change, so the cache is filled after its first lambda)
    bool moved = l0 > 0;
    if (grp) {
        for (int g = threadIdx.x; g < P.ngroups; g += kStreamThreads)
            for (int q = gstart[g]; q < gstart[g + 1]; ++q) S.gof[gidx[q]] = g;
    }

    // publish this wave's nonzero coefficients into list buffer `buf`: cached
    // coordinates write their value (zero included) to their slot, the other
    // nonzero ones go to the wave's list segment
    auto publish = [&](int buf) {
        int base = 0;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            if (myslot[r] >= 0) S.cb[buf * kCacheMax + myslot[r]] = bt[r];
            const bool nz = mine[r] && bt[r] != 0.0 && myslot[r] < 0;
            const uint64_t ball = __ballot(nz);
            if (nz) {
                const int k = base + __popcll(ball & ((1ull << lane) - 1ull));
                S.lj[(buf * NW + wave) * SEG + k] = row[r];
                S.lb[(buf * NW + wave) * SEG + k] = bt[r];
            }
            base += __popcll(ball);
        }
        if (lane == 0) S.lcnt[buf * NW + wave] = base;
    };
    // G beta for this lane's coordinates from list buffer `buf`.  The eight
    // segments are read as one list of `total` entries, 64 entries per chunk
    // (lane k holds entry k); within a chunk the loads of 2 U entries are
    // issued before their products, so each lane keeps 2 U R row-segment
    // loads in flight.  Entries past the end read as (column 0, value 0).
    auto matvec = [&](int buf, double (&gb)[R]) {
        constexpr int U = R == 1 ? 16 : (R == 2 ? 4 : 2);
        int pref[NW + 1];
        pref[0] = 0;
#pragma unroll
        for (int w = 0; w < NW; ++w)
            pref[w + 1] = pref[w] + __builtin_amdgcn_readfirstlane(S.lcnt[buf * NW + w]);
        const int total = pref[NW];
        double acc[R][4];
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
            for (int a = 0; a < 4; ++a) acc[r][a] = 0.0;
        int rc[R];
#pragma unroll
        for (int r = 0; r < R; ++r) rc[r] = mine[r] ? row[r] : 0;
        // cached columns from LDS (slots past ncached read as value 0)
        if (ncached > 0) {
            const double cv = lane < ncached ? S.cb[buf * kCacheMax + lane] : 0.0;
            const int clo = __double2loint(cv), chi = __double2hiint(cv);
            constexpr int UC = R == 1 ? 8 : 4;
            for (int e0 = 0; e0 < ncached; e0 += UC) {
                double gv[UC][R], bj[UC];
#pragma unroll
                for (int u = 0; u < UC; ++u) {
                    const int e = min(e0 + u, 63);
                    const int sl = min(e0 + u, ncached - 1);
                    bj[u] = (e0 + u < ncached) ? __hiloint2double(__builtin_amdgcn_readlane(chi, e),
                                                                  __builtin_amdgcn_readlane(clo, e))
                                               : 0.0;
#pragma unroll
                    for (int r = 0; r < R; ++r) gv[u][r] = S.cache[(size_t)sl * p + rc[r]];
                }
#pragma unroll
                for (int u = 0; u < UC; ++u)
#pragma unroll
                    for (int r = 0; r < R; ++r) acc[r][u % 4] += gv[u][r] * bj[u];
            }
        }
        for (int cb = 0; cb < total; cb += 64) {
            const int idx = cb + lane;
            int sg = 0;
#pragma unroll
            for (int w = 1; w < NW; ++w) sg += (idx >= pref[w]) ? 1 : 0;
            const bool ok = idx < total;
            const int off = ok ? (buf * NW + sg) * SEG + (idx - pref[sg]) : 0;
            const int jv = ok ? S.lj[off] : 0;
            const double bv = ok ? S.lb[off] : 0.0;
            const int m = min(64, total - cb);
            const int blo = __double2loint(bv), bhi = __double2hiint(bv);
            for (int e0 = 0; e0 < m; e0 += 2 * U) {
                double gv[2 * U][R], bj[2 * U];
#pragma unroll
                for (int u = 0; u < 2 * U; ++u) {
                    const int e = min(e0 + u, 63);
                    const int j = __builtin_amdgcn_readlane(jv, e);
                    bj[u] = (e0 + u < m) ? __hiloint2double(__builtin_amdgcn_readlane(bhi, e),
                                                            __builtin_amdgcn_readlane(blo, e))
                                         : 0.0;
                    const auto gcol = Gg + (size_t)j * p;
#pragma unroll
                    for (int r = 0; r < R; ++r) gv[u][r] = gcol[rc[r]];
                }
#pragma unroll
                for (int u = 0; u < 2 * U; ++u)
#pragma unroll
                    for (int r = 0; r < R; ++r) acc[r][u % 4] += gv[u][r] * bj[u];
            }
        }
#pragma unroll
        for (int r = 0; r < R; ++r) gb[r] = (acc[r][0] + acc[r][1]) + (acc[r][2] + acc[r][3]);
    };

    int cur = 0;
    publish(cur);
    __syncthreads();
    double gb[R];
    matvec(cur, gb);

    for (int l = l0; l < P.L; ++l) {
        const double lam = lambda_g[l];
        Upd q[R];
#pragma unroll
        for (int r = 0; r < R; ++r) q[r] = make_upd(P.kind, wt[r] * lam, d, P.alpha, P.gamma);
        int it = 0;
        bool conv = false;
        do {
            double dl = 0.0, mx = 0.0;
            double u[R];
#pragma unroll
            for (int r = 0; r < R; ++r) u[r] = ct[r] + (d * bt[r] - gb[r]);
            if (grp) {
#pragma unroll
                for (int r = 0; r < R; ++r)
                    if (mine[r]) S.us[row[r]] = u[r];
                __syncthreads();
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    if (!mine[r]) continue;
                    const int g = S.gof[row[r]];
                    double ss = 0.0;
                    for (int qq = gstart[g]; qq < gstart[g + 1]; ++qq) {
                        const double v = S.us[gidx[qq]];
                        ss += v * v;
                    }
                    const double nrm = sqrt(ss);
                    const double f = nrm > 0.0 ? 1.0 - cgw[g] * lam / nrm : 0.0;
                    const double bn = f > 0.0 ? (u[r] * inv_d) * f : 0.0;
                    moved |= (bn == 0.0) != (bt[r] == 0.0);
                    dl = nmax(dl, fabs(bn - bt[r]));
                    mx = nmax(mx, fabs(bn));
                    bt[r] = bn;
                }
            } else {
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    if (!mine[r]) continue;
                    const double bn = update_fast(P.kind, u[r], q[r], P.gamma);
                    moved |= (bn == 0.0) != (bt[r] == 0.0);
                    dl = nmax(dl, fabs(bn - bt[r]));
                    mx = nmax(mx, fabs(bn));
                    bt[r] = bn;
                }
            }
            ++it;
            dl = lanes_max<64>(dl);
            mx = lanes_max<64>(mx);
            const int nxt = cur ^ 1;
            publish(nxt);
            if (lane == 0) {
                S.dm[(nxt * NW + wave) * 2] = dl;
                S.dm[(nxt * NW + wave) * 2 + 1] = mx;
            }
            __syncthreads();
            cur = nxt;
            matvec(cur, gb);
            double DL = S.dm[cur * NW * 2], MX = S.dm[cur * NW * 2 + 1];
#pragma unroll
            for (int w = 1; w < NW; ++w) {
                DL = nmax(DL, S.dm[(cur * NW + w) * 2]);
                MX = nmax(MX, S.dm[(cur * NW + w) * 2 + 1]);
            }
            conv = DL <= P.tol * MX;
        } while (!conv && it < P.maxit);

        // stationarity and objective at the accepted beta (gb = G beta)
        double kv = 0.0, penv = 0.0, quad = 0.0, lin = 0.0;
        if (grp) {
#pragma unroll
            for (int r = 0; r < R; ++r)
                if (mine[r]) S.us[row[r]] = gb[r] - ct[r];     // gradient
            __syncthreads();
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
            if (!mine[r]) continue;
            quad += bt[r] * gb[r];
            lin += ct[r] * bt[r];
            if (!grp) {
                const double lw = wt[r] * lam;
                const double g = gb[r] - ct[r];
                if (bt[r] == 0.0)
                    kv = nmax(kv, pos(fabs(g) - (P.kind == OEM_ENET ? P.alpha * lw : lw)));
                else
                    kv = nmax(kv, fabs(g + sgn(bt[r]) * pen_deriv(P.kind, fabs(bt[r]), lw, P.alpha, P.gamma)));
                penv += pen_value(P.kind, bt[r], lw, P.alpha, P.gamma);
            }
        }
        if (grp) {
            // group KKT and penalty need beta of every member: stage beta in LDS
            __syncthreads();
            double *bs = S.lb;     // list buffers are free until the next publish
#pragma unroll
            for (int r = 0; r < R; ++r)
                if (mine[r]) bs[row[r]] = bt[r];
            __syncthreads();
#pragma unroll
            for (int r = 0; r < R; ++r) {
                if (!mine[r]) continue;
                const int g = S.gof[row[r]];
                const int q0 = gstart[g], q1 = gstart[g + 1];
                if (gidx[q0] != row[r]) continue;
                const double lc = lam * cgw[g];
                double bn = 0.0, gn = 0.0;
                for (int qq = q0; qq < q1; ++qq) {
                    const int j = gidx[qq];
                    bn += bs[j] * bs[j];
                    gn += S.us[j] * S.us[j];
                }
                bn = sqrt(bn);
                gn = sqrt(gn);
                double v;
                if (bn > 0.0) {
                    double ss = 0.0;
                    for (int qq = q0; qq < q1; ++qq) {
                        const int j = gidx[qq];
                        const double rr = S.us[j] + lc * bs[j] / bn;
                        ss += rr * rr;
                    }
                    v = sqrt(ss);
                } else {
                    v = pos(gn - lc);
                }
                kv = nmax(kv, v);
                penv += lc * bn;
            }
        }
        kv = wave_max(kv);
        penv = wave_sum(penv);
        quad = wave_sum(quad);
        lin = wave_sum(lin);
        const bool wmoved = __ballot(moved) != 0;
        if (lane == 0) {
            S.fin[0 * NW + wave] = kv;
            S.fin[1 * NW + wave] = penv;
            S.fin[2 * NW + wave] = quad;
            S.fin[3 * NW + wave] = lin;
            S.wcnt[wave] = wmoved ? 1 : 0;
        }
        __syncthreads();
        bool refill = false;
#pragma unroll
        for (int w = 0; w < NW; ++w) refill |= S.wcnt[w] != 0;
        if (threadIdx.x == 0) {
            kv = S.fin[0];
            penv = S.fin[NW];
            quad = S.fin[2 * NW];
            lin = S.fin[3 * NW];
            for (int w = 1; w < NW; ++w) {
                kv = nmax(kv, S.fin[w]);
                penv += S.fin[NW + w];
                quad += S.fin[2 * NW + w];
                lin += S.fin[3 * NW + w];
            }
            if (kkt_g) kkt_g[l] = kv;
            if (obj_g) obj_g[l] = 0.5 * quad - lin + 0.5 * yyn + penv;
            if (iters_g) iters_g[l] = conv ? it : -it;
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
            if (!mine[r]) continue;
            beta_g[(size_t)l * p + row[r]] = bt[r] / st[r];
            if (beta_std_g) beta_std_g[(size_t)l * p + row[r]] = bt[r];
        }
        if (grp) {
            // the staged beta overwrote list buffers: publish the current
            // list again so the next lambda starts from a consistent state
            __syncthreads();
            publish(cur);
            __syncthreads();
        }
        // the support changed during this lambda: give the cache slots to the
        // first nonzero coordinates (wave order, then r, then lane) and load
        // their columns; the G beta carried into the next lambda is unchanged
        if (refill && cache_cols > 0) {
            __syncthreads();                       // flags in S.wcnt are read
            int wc = 0;
            uint64_t ball[R];
#pragma unroll
            for (int r = 0; r < R; ++r) {
                ball[r] = __ballot(mine[r] && bt[r] != 0.0);
                wc += __popcll(ball[r]);
            }
            if (lane == 0) S.wcnt[wave] = wc;
            __syncthreads();
            int off = 0, total = 0;
            for (int w = 0; w < NW; ++w) {
                off += (w < wave) ? S.wcnt[w] : 0;
                total += S.wcnt[w];
            }
            int pos = off;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const bool nz = (ball[r] >> lane) & 1ull;
                const int at = pos + __popcll(ball[r] & ((1ull << lane) - 1ull));
                myslot[r] = (nz && at < cache_cols) ? at : -1;
                if (myslot[r] >= 0) S.cj[at] = row[r];
                pos += __popcll(ball[r]);
            }
            ncached = min(total, cache_cols);
            __syncthreads();
            for (int e = threadIdx.x; e < ncached * p; e += kStreamThreads) {
                const int sl = e / p, i = e - sl * p;
                S.cache[(size_t)sl * p + i] = Gg[(size_t)S.cj[sl] * p + i];
            }
            __syncthreads();
        }
        moved = false;
    }
}

int launch_paths_stream(const PathDesc *d_desc, const int *d_order, int count, int pmax, int chain,
                        hipStream_t s)
{
    if (count == 0) return OEM_OK;
    const void *kern;
    int R;
    if (pmax <= 512) {
        kern = (const void *)path_stream_kernel<1>;
        R = 1;
    } else if (pmax <= 1024) {
        kern = (const void *)path_stream_kernel<2>;
        R = 2;
    } else if (pmax <= 2048) {
        kern = (const void *)path_stream_kernel<4>;
        R = 4;
    } else {
        return fail(OEM_E_INVAL, "streaming path kernel needs p <= 2048");
    }
    int cols = path_stream_cache_cols(R, pmax);
    const size_t lds = path_stream_lds_bytes(R, pmax, cols);
    OEM_HIP_CHECK(hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    void *args[] = {(void *)&d_desc, (void *)&d_order, (void *)&cols, (void *)&chain};
    OEM_HIP_CHECK(hipLaunchKernel(kern, dim3(count), dim3(kStreamThreads), args, lds, s));
    return OEM_OK;
}

} // namespace oem
