// OEM lambda paths (Section 2.1 iteration, Section 2.2 updates), lambda grids
// and cross-validation error (Section 3).
//
// One workgroup runs one whole warm-started path: for each lambda it repeats
//     u = c + (d I - G) beta          (only columns with beta_j != 0 are read)
//     beta <- update(u)               (thresholding operator of the penalty)
// until max|delta beta| <= tol * max|beta|.  G is kept in LDS when it fits,
// otherwise it streams from L2.  Every (problem, fold, penalty) path is
// independent, so paths of different problems and sizes share one launch.
#include <algorithm>
#include <cstdlib>

#include "path_common.h"

namespace oem {

// ---------------------------------------------------------------- lambda grid

// Sparse group lasso: does the update map beta = 0 (u = cs) of the group
// with members gidx[t0..t1) to a nonzero vector at lambda?
__device__ inline bool sgl_group_nonzero(const double *cs, const int32_t *gidx, int t0, int t1,
                                         const double *w, double cgk, double tau, double lam)
{
    double ss = 0.0;
    for (int t = t0; t < t1; ++t) {
        const int j = gidx[t];
        const double v = pos(fabs(cs[j]) - (w ? w[j] : 1.0) * lam * tau);
        ss += v * v;
    }
    const double nrm = sqrt(ss);
    return nrm > 0.0 && 1.0 - cgk * lam * (1.0 - tau) / nrm > 0.0;
}

// Smallest lambda that zeroes the group: for tau = 1 each penalised
// member's lasso threshold; otherwise ||soft(c_g, w lambda tau)|| - c lambda
// (1 - tau) decreases in lambda and is <= 0 at ||c_g|| / (c (1 - tau)), and
// the crossing is bisected over doubles down to adjacent values.
__device__ inline double sgl_group_lambda_max(const double *cs, const int32_t *gidx, int t0, int t1,
                                              const double *w, double cgk, double tau)
{
    if (tau >= 1.0) {
        double lg = 0.0;
        for (int t = t0; t < t1; ++t) {
            const int j = gidx[t];
            const double wj = w ? w[j] : 1.0;
            if (wj <= 0.0) continue;
            double lj = fabs(cs[j]) / wj;
            while (fabs(cs[j]) - wj * lj > 0.0) lj = nextafter(lj, INFINITY);
            lg = fmax(lg, lj);
        }
        return lg;
    }
    double ss = 0.0;
    for (int t = t0; t < t1; ++t) ss += cs[gidx[t]] * cs[gidx[t]];
    double lo = 0.0, hi = sqrt(ss) / (cgk * (1.0 - tau));
    if (!sgl_group_nonzero(cs, gidx, t0, t1, w, cgk, tau, lo)) return 0.0;
    while (sgl_group_nonzero(cs, gidx, t0, t1, w, cgk, tau, hi)) hi = nextafter(hi, INFINITY);
    for (;;) {
        const double mid = lo + 0.5 * (hi - lo);
        if (!(mid > lo && mid < hi)) break;
        if (sgl_group_nonzero(cs, gidx, t0, t1, w, cgk, tau, mid))
            lo = mid;
        else
            hi = mid;
    }
    return hi;
}

// lambda_max of penalty `pen` from the full-data standardised X^T y: the
// smallest value at which the update maps beta = 0 to 0 (each candidate is
// raised by ulps until the update's own zero test holds), then a log grid.
__global__ __launch_bounds__(kPathThreads) void lambda_grid_kernel(
    const double *__restrict__ cs, int p, const int32_t *__restrict__ gstart,
    const int32_t *__restrict__ gidx, int ngroups, const double *__restrict__ w,
    const double *__restrict__ cg, const oem_penalty *__restrict__ pens, int L, double ratio,
    double *__restrict__ lambda_out)
{
    __shared__ double red[kPathWaves];
    const oem_penalty pen = pens[blockIdx.x];
    double m = 0.0;
    if (pen.kind == OEM_SGL) {
        for (int gi = threadIdx.x; gi < ngroups; gi += kPathThreads)
            m = fmax(m, sgl_group_lambda_max(cs, gidx, gstart[gi], gstart[gi + 1], w, cg[gi], pen.tau));
    } else if (group_penalty(pen.kind)) {
        for (int gi = threadIdx.x; gi < ngroups; gi += kPathThreads) {
            double ss = 0.0;
            for (int t = gstart[gi]; t < gstart[gi + 1]; ++t) ss += cs[gidx[t]] * cs[gidx[t]];
            const double nrm = sqrt(ss), c = cg[gi];
            double lg = nrm / c;
            // the update's own zero test: the group lasso factor, or the
            // soft part of the MCP / SCAD update of ||u||
            if (pen.kind == OEM_GRP_LASSO)
                while (nrm > 0.0 && 1.0 - c * lg / nrm > 0.0) lg = nextafter(lg, INFINITY);
            else
                while (nrm - c * lg > 0.0) lg = nextafter(lg, INFINITY);
            m = fmax(m, lg);
        }
    } else {
        const double a = pen.kind == OEM_ENET ? pen.alpha : 1.0;
        for (int j = threadIdx.x; j < p; j += kPathThreads) {
            const double wj = w ? w[j] : 1.0;
            if (wj <= 0.0) continue;
            const double ac = fabs(cs[j]);
            double lj = ac / (wj * a);
            if (pen.kind == OEM_ENET) {
                while (ac - wj * lj * a > 0.0) lj = nextafter(lj, INFINITY);
            } else {
                while (ac - wj * lj > 0.0) lj = nextafter(lj, INFINITY);
            }
            m = fmax(m, lj);
        }
    }
    m = wave_max(m);
    if (threadIdx.x % kWave == 0) red[threadIdx.x / kWave] = m;
    __syncthreads();
    double lmax = red[0];
    for (int i = 1; i < kPathWaves; ++i) lmax = fmax(lmax, red[i]);
    for (int l = threadIdx.x; l < L; l += kPathThreads)
        lambda_out[(size_t)blockIdx.x * L + l] =
            (L == 1) ? lmax : lmax * pow(ratio, (double)l / (double)(L - 1));
}

// ---------------------------------------------------------------- path kernel

struct PathLds {
    double *beta, *u, *Gl;
    int *act;
    double *red;
    int *iscan;
};

// u = c + (d beta - G beta) over the active columns; also returns nothing.
__device__ inline void oem_u(const PathDesc &P, const double *G, int ldg, const PathLds &S,
                             int nact, double d)
{
    const int p = P.p;
    for (int i = threadIdx.x; i < p; i += kPathThreads) {
        double acc = 0.0;
        int a = 0;
        for (; a + 4 <= nact; a += 4) {
            const int j0 = S.act[a], j1 = S.act[a + 1], j2 = S.act[a + 2], j3 = S.act[a + 3];
            acc += G[(size_t)j0 * ldg + i] * S.beta[j0];
            acc += G[(size_t)j1 * ldg + i] * S.beta[j1];
            acc += G[(size_t)j2 * ldg + i] * S.beta[j2];
            acc += G[(size_t)j3 * ldg + i] * S.beta[j3];
        }
        for (; a < nact; ++a) {
            const int j = S.act[a];
            acc += G[(size_t)j * ldg + i] * S.beta[j];
        }
        S.u[i] = P.c[i] + (d * S.beta[i] - acc);
    }
}

// ordered list of nonzero coordinates; returns the count (uniform)
__device__ inline int rebuild_active(const PathLds &S, int p)
{
    const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
    int base = 0;
    for (int i0 = 0; i0 < p; i0 += kPathThreads) {
        const int i = i0 + threadIdx.x;
        const int nz = (i < p) && (S.beta[i] != 0.0);
        const uint64_t ball = __ballot(nz);
        const int before = __popcll(ball & ((1ull << lane) - 1ull));
        if (lane == 0) S.iscan[wave] = __popcll(ball);
        __syncthreads();
        int off = 0, tot = 0;
        for (int w = 0; w < kPathWaves; ++w) {
            if (w < wave) off += S.iscan[w];
            tot += S.iscan[w];
        }
        if (nz) S.act[base + off + before] = i;
        __syncthreads();
        base += tot;
    }
    return base;
}

__global__ __launch_bounds__(kPathThreads) void path_kernel(const PathDesc *__restrict__ descs,
                                                            const int *__restrict__ order,
                                                            int lds_g_max_p)
{
    extern __shared__ double sm[];
    const PathDesc P = descs[order ? order[blockIdx.x] : blockIdx.x];
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
    const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
    PathLds S;
    S.beta = sm;
    S.u = S.beta + p;
    S.red = S.u + p;                               // 4 * kPathWaves + 2
    S.act = reinterpret_cast<int *>(S.red + 4 * kPathWaves + 2);
    S.iscan = S.act + p + 1;                       // kPathWaves
    double *after_ints = sm + 2 * p + 4 * kPathWaves + 2 + (p + 1 + kPathWaves + 1) / 2 + 1;
    const bool g_in_lds = p <= lds_g_max_p;
    const double *G = P.G;   // G may move to LDS below: generic pointer
    if (g_in_lds) {
        S.Gl = after_ints;
        for (size_t e = threadIdx.x; e < (size_t)p * p; e += kPathThreads) S.Gl[e] = G_g[e];
        G = S.Gl;
    }
    const double d = *P.d;
    const double yyn = *P.yyn;
    const bool grp = group_penalty(P.kind);
    const auto init_g = gmem(P.beta_init);
    for (int i = threadIdx.x; i < p; i += kPathThreads) S.beta[i] = P.beta_init ? init_g[i] : 0.0;
    __syncthreads();
    int nact = P.beta_init ? rebuild_active(S, p) : 0;

    for (int l = 0; l < P.L; ++l) {
        const double lam = lambda_g[l];
        int it = 0;
        bool conv = false;
        while (it < P.maxit) {
            oem_u(P, G, p, S, nact, d);
            __syncthreads();
            // update, change and size
            double dl = 0.0, mx = 0.0;
            if (grp) {
                for (int gi = threadIdx.x; gi < P.ngroups; gi += kPathThreads) {
                    double ss = 0.0;
                    const int t0 = gstart_g[gi], t1 = gstart_g[gi + 1];
                    if (P.kind == OEM_SGL) {
                        // inner soft threshold first (nested penalties), in place of u
                        for (int t = t0; t < t1; ++t) {
                            const int j = gidx_g[t];
                            const double v = sgl_inner(S.u[j], w_g ? w_g[j] : 1.0, lam, P.tau);
                            S.u[j] = v;
                            ss += v * v;
                        }
                    } else {
                        for (int t = t0; t < t1; ++t) ss += S.u[gidx_g[t]] * S.u[gidx_g[t]];
                    }
                    const double nrm = sqrt(ss);
                    const GroupUpd gu =
                        make_group_upd(P.kind, nrm, group_lam_c(P.kind, cg_g[gi], lam, P.tau), d, P.gamma);
                    for (int t = t0; t < t1; ++t) {
                        const int j = gidx_g[t];
                        const double bn = group_update_one(gu, S.u[j]);
                        dl = fmax(dl, fabs(bn - S.beta[j]));
                        mx = fmax(mx, fabs(bn));
                        S.beta[j] = bn;
                    }
                }
            } else {
                for (int i = threadIdx.x; i < p; i += kPathThreads) {
                    const double lw = (w_g ? w_g[i] : 1.0) * lam;
                    const double bn = update1(P.kind, S.u[i], lw, d, P.alpha, P.gamma);
                    dl = fmax(dl, fabs(bn - S.beta[i]));
                    mx = fmax(mx, fabs(bn));
                    S.beta[i] = bn;
                }
            }
            dl = wave_max(dl);
            mx = wave_max(mx);
            if (lane == 0) {
                S.red[wave] = dl;
                S.red[kPathWaves + wave] = mx;
            }
            __syncthreads();
            dl = S.red[0];
            mx = S.red[kPathWaves];
            for (int wv = 1; wv < kPathWaves; ++wv) {
                dl = fmax(dl, S.red[wv]);
                mx = fmax(mx, S.red[kPathWaves + wv]);
            }
            nact = rebuild_active(S, p);
            ++it;
            if (dl <= P.tol * mx) {
                conv = true;
                break;
            }
        }
        // gradient g = G beta - c, stationarity and objective (FP64)
        double kv = 0.0, quad = 0.0, lin = 0.0, penv = 0.0;
        for (int i = threadIdx.x; i < p; i += kPathThreads) {
            double acc = 0.0;
            for (int a = 0; a < nact; ++a) {
                const int j = S.act[a];
                acc += G[(size_t)j * p + i] * S.beta[j];
            }
            S.u[i] = acc - c_g[i];   // gradient
            quad += S.beta[i] * acc;
            lin += c_g[i] * S.beta[i];
            if (!grp) {
                const double lw = (w_g ? w_g[i] : 1.0) * lam;
                const double b = S.beta[i];
                double v;
                if (b == 0.0) {
                    v = pos(fabs(S.u[i]) - (P.kind == OEM_ENET ? P.alpha * lw : lw));
                } else {
                    v = fabs(S.u[i] + sgn(b) * pen_deriv(P.kind, fabs(b), lw, P.alpha, P.gamma));
                }
                kv = fmax(kv, v);
                penv += pen_value(P.kind, b, lw, P.alpha, P.gamma);
            }
        }
        __syncthreads();
        if (grp) {
            for (int gi = threadIdx.x; gi < P.ngroups; gi += kPathThreads) {
                const double cgk = cg_g[gi];
                const double lc = group_lam_c(P.kind, cgk, lam, P.tau);
                double bn = 0.0, gn = 0.0, l1w = 0.0;
                const int t0 = gstart_g[gi], t1 = gstart_g[gi + 1];
                for (int t = t0; t < t1; ++t) {
                    const int j = gidx_g[t];
                    bn += S.beta[j] * S.beta[j];
                    gn += S.u[j] * S.u[j];
                    l1w += (w_g ? w_g[j] : 1.0) * fabs(S.beta[j]);
                }
                bn = sqrt(bn);
                gn = sqrt(gn);
                double v;
                if (P.kind == OEM_SGL) {
                    // 0 in g + lambda (1 - tau) c dN(beta_g) + lambda tau w d|beta|:
                    // a zero group is stationary when ||soft(g, lambda tau w)|| <= lc
                    double ss = 0.0;
                    for (int t = t0; t < t1; ++t) {
                        const int j = gidx_g[t];
                        const double lt = lam * P.tau * (w_g ? w_g[j] : 1.0);
                        const double r = (bn == 0.0 || S.beta[j] == 0.0)
                                             ? pos(fabs(S.u[j]) - lt)
                                             : S.u[j] + lc * S.beta[j] / bn + lt * sgn(S.beta[j]);
                        ss += r * r;
                    }
                    v = bn == 0.0 ? pos(sqrt(ss) - lc) : sqrt(ss);
                } else if (bn > 0.0) {
                    const double dp = group_pen_deriv(P.kind, bn, lc, P.gamma);
                    double ss = 0.0;
                    for (int t = t0; t < t1; ++t) {
                        const int j = gidx_g[t];
                        const double r = S.u[j] + dp * S.beta[j] / bn;
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
        quad = wave_sum(quad);
        lin = wave_sum(lin);
        penv = wave_sum(penv);
        __syncthreads();
        if (lane == 0) {
            S.red[wave] = kv;
            S.red[kPathWaves + wave] = quad;
            S.red[2 * kPathWaves + wave] = lin;
            S.red[3 * kPathWaves + wave] = penv;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            double k2 = 0.0, q2 = 0.0, l2 = 0.0, p2 = 0.0;
            for (int wv = 0; wv < kPathWaves; ++wv) {
                k2 = fmax(k2, S.red[wv]);
                q2 += S.red[kPathWaves + wv];
                l2 += S.red[2 * kPathWaves + wv];
                p2 += S.red[3 * kPathWaves + wv];
            }
            if (kkt_g) kkt_g[l] = k2;
            if (obj_g) obj_g[l] = 0.5 * q2 - l2 + 0.5 * yyn + p2;
            if (iters_g) iters_g[l] = conv ? it : -it;
        }
        for (int i = threadIdx.x; i < p; i += kPathThreads) {
            beta_g[(size_t)l * p + i] = S.beta[i] / s_g[i];
            if (beta_std_g) beta_std_g[(size_t)l * p + i] = S.beta[i];
        }
        __syncthreads();
    }
}

size_t path_lds_bytes(int p, bool g_in_lds)
{
    size_t doubles = 2 * (size_t)p + 4 * kPathWaves + 2 + ((size_t)p + 1 + kPathWaves + 1) / 2 + 1;
    if (g_in_lds) doubles += (size_t)p * p;
    return doubles * sizeof(double);
}

int launch_paths_reg(const PathDesc *d_desc, const int *d_order, int count, int pmax, int chain,
                     hipStream_t s);
int launch_paths_blk(const PathDesc *d_desc, const int *d_order, int count, int pmax, int chain,
                     hipStream_t s);
int launch_paths_stream(const PathDesc *d_desc, const int *d_order, int count, int pmax, int chain,
                        hipStream_t s);
int launch_paths_ws(const PathDesc *d_desc, const int *d_order, int count, int nw, int first, int pmax,
                    hipStream_t s);

// Path kernels: 0..2 block kernel (separable penalties, p <= 32, 64, 128),
// 3, 4 register kernel (group lasso, p <= 64, 128), 5 streaming kernel
// (128 < p <= 2048), 6 general kernel (larger p), 7, 8, 9 working-set kernel
// on 1, 2, 4 waves.
enum { kBlk32, kBlk64, kBlk128, kReg64, kReg128, kStream, kGeneral, kWs1, kWs2, kWs4 };

// Launch slots in enqueue order: (kernel, continues an earlier launch).  A
// path's launches are always enqueued in the order of its chain, and a
// kernel reads the hand-over only in a slot marked as continuing.
struct PathSlot {
    int kernel, chain;
};
static const PathSlot kSlots[] = {
    {kWs1, 0},    {kWs2, 0},     {kWs2, 1},    {kWs4, 1},    {kBlk32, 0},   {kBlk64, 0},
    {kBlk128, 0}, {kReg64, 0},   {kReg128, 0}, {kStream, 0}, {kBlk64, 1},   {kBlk128, 1},
    {kReg64, 1},  {kReg128, 1},  {kStream, 1}, {kGeneral, 0}};
constexpr int kNumSlots = sizeof(kSlots) / sizeof(kSlots[0]);

static int slot_index(int kernel, int chain)
{
    for (int i = 0; i < kNumSlots; ++i)
        if (kSlots[i].kernel == kernel && kSlots[i].chain == chain) return i;
    return -1;
}

// The working-set kernels can be switched off (OEM_PATH_WS=0) to run every
// path on its kernel class alone.
static bool ws_enabled()
{
    static const bool on = [] {
        const char *e = getenv("OEM_PATH_WS");
        return !(e && e[0] == '0');
    }();
    return on;
}

// Launch slots of one path, in order.  Separable penalties at p <= 32 run on
// the block kernel alone; larger p start on a working-set kernel of 1 or 2
// waves, continue on one of 2 or 4 waves when the working set outgrows it,
// and end on the kernel of their class; p > 2048 runs on the general kernel.
static int path_chain(const PathDesc &d, int *slots)
{
    const bool grp = d.kind == OEM_GRP_LASSO;
    // group MCP, group SCAD and the sparse group lasso run on the general kernel
    const int cls = (d.p > 2048 || (group_penalty(d.kind) && !grp) || d.beta_init) ? kGeneral
                    : d.p > 128 ? kStream
                    : grp       ? (d.p <= 64 ? kReg64 : kReg128)
                                : (d.p <= 32 ? kBlk32 : (d.p <= 64 ? kBlk64 : kBlk128));
    int n = 0;
    if (cls == kGeneral || cls == kBlk32 || !ws_enabled()) {
        slots[n++] = slot_index(cls, 0);
        return n;
    }
    if (d.p <= 128) {
        slots[n++] = slot_index(kWs1, 0);
        if (d.p > 64) slots[n++] = slot_index(kWs2, 1);
    } else {
        slots[n++] = slot_index(kWs2, 0);
        slots[n++] = slot_index(kWs4, 1);
    }
    slots[n++] = slot_index(cls, 1);
    return n;
}

void plan_paths(const std::vector<PathDesc> &host, PathPlan &plan)
{
    plan.order.clear();
    plan.launches.clear();
    std::vector<std::vector<int>> by_slot(kNumSlots);
    for (int i = 0; i < (int)host.size(); ++i) {
        int sl[4];
        const int n = path_chain(host[i], sl);
        for (int k = 0; k < n; ++k) by_slot[sl[k]].push_back(i);
    }
    for (int c = 0; c < kNumSlots; ++c) {
        if (by_slot[c].empty()) continue;
        const int first = (int)plan.order.size();
        int pmax = 0;
        for (int i : by_slot[c]) {
            plan.order.push_back(i);
            pmax = std::max(pmax, host[i].p);
        }
        plan.launches.push_back(PathLaunch{c, first, (int)by_slot[c].size(), pmax, kSlots[c].chain});
    }
}

int attach_path_handover(std::vector<PathDesc> &descs, DevBuf &buf)
{
    size_t bytes = 0;
    for (const PathDesc &d : descs) bytes += sizeof(double) * (1 + (size_t)d.p);
    int rc = buf.ensure(std::max<size_t>(bytes, 64));
    if (rc) return rc;
    char *base = buf.as<char>();
    size_t off = 0;
    for (PathDesc &d : descs) {
        d.lstart = reinterpret_cast<int32_t *>(base + off);
        d.bws = reinterpret_cast<double *>(base + off + sizeof(double));
        off += sizeof(double) * (1 + (size_t)d.p);
    }
    return OEM_OK;
}

static int launch_general(const PathDesc *d_desc, const int *ord, int count, int pmax, hipStream_t s);

int launch_paths_planned(const PathDesc *d_desc, const int *d_order, const PathPlan &plan,
                         hipStream_t s)
{
    for (const PathLaunch &L : plan.launches) {
        const int *ord = d_order + L.first;
        const int ch = L.chain;
        int rc = OEM_OK;
        switch (kSlots[L.cls].kernel) {
        case kWs1: rc = launch_paths_ws(d_desc, ord, L.count, 1, !ch, L.pmax, s); break;
        case kWs2: rc = launch_paths_ws(d_desc, ord, L.count, 2, !ch, L.pmax, s); break;
        case kWs4: rc = launch_paths_ws(d_desc, ord, L.count, 4, !ch, L.pmax, s); break;
        case kBlk32: rc = launch_paths_blk(d_desc, ord, L.count, 32, ch, s); break;
        case kBlk64: rc = launch_paths_blk(d_desc, ord, L.count, 64, ch, s); break;
        case kBlk128: rc = launch_paths_blk(d_desc, ord, L.count, 128, ch, s); break;
        case kReg64: rc = launch_paths_reg(d_desc, ord, L.count, 64, ch, s); break;
        case kReg128: rc = launch_paths_reg(d_desc, ord, L.count, 128, ch, s); break;
        case kStream: rc = launch_paths_stream(d_desc, ord, L.count, L.pmax, ch, s); break;
        default: rc = launch_general(d_desc, ord, L.count, L.pmax, s); break;
        }
        if (rc) return rc;
    }
    return OEM_OK;
}

static int launch_general(const PathDesc *d_desc, const int *ord, int count, int pmax, hipStream_t s)
{
    // keep G in LDS when the largest path's matrix fits next to its vectors
    const size_t limit = 150 * 1024;
    int lds_g_max_p = 0;
    size_t lds = path_lds_bytes(pmax, false);
    if (path_lds_bytes(pmax, true) <= limit) {
        lds_g_max_p = pmax;
        lds = path_lds_bytes(pmax, true);
    }
    OEM_HIP_CHECK(hipFuncSetAttribute((const void *)path_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                      (int)lds));
    hipLaunchKernelGGL(path_kernel, dim3(count), dim3(kPathThreads), lds, s, d_desc, ord, lds_g_max_p);
    OEM_HIP_CHECK(hipGetLastError());
    return OEM_OK;
}

int launch_paths_general(const PathDesc *d_desc, int count, int pmax, hipStream_t s)
{
    return count > 0 ? launch_general(d_desc, nullptr, count, pmax, s) : OEM_OK;
}

// One set of launches for paths of any p: the order table groups the paths
// by kernel class.
int launch_paths(const PathDesc *d_desc, const std::vector<PathDesc> &host, DevBuf &orderbuf,
                 hipStream_t s, oem_gram_s *stage_owner)
{
    if (host.empty()) return OEM_OK;
    PathPlan plan;
    plan_paths(host, plan);
    int rc = orderbuf.ensure(plan.order.size() * sizeof(int));
    if (rc) return rc;
    rc = stage_upload(stage_owner, kUpOrder, orderbuf.ptr, plan.order.data(), plan.order.size() * sizeof(int), s);
    if (rc) return rc;
    return launch_paths_planned(d_desc, orderbuf.as<int>(), plan, s);
}

int launch_lambda_grid(const double *cs_full, int p, const int32_t *gstart, const int32_t *gidx,
                       int ngroups, const double *w, const double *cg, const oem_penalty *d_pens,
                       int npen, int L, double ratio, double *lambda_out, hipStream_t s)
{
    hipLaunchKernelGGL(lambda_grid_kernel, dim3(npen), dim3(kPathThreads), 0, s, cs_full, p, gstart,
                       gidx, ngroups, w, cg, d_pens, L, ratio, lambda_out);
    OEM_HIP_CHECK(hipGetLastError());
    return OEM_OK;
}

// ---------------------------------------------------------------- intercepts

// beta0_l = ybar - xbar^T beta_l (original scale), the unpenalised intercept
// of a centred problem; one workgroup per path, sums in a fixed order.
__global__ __launch_bounds__(kPathThreads) void intercept_kernel(const PathDesc *__restrict__ descs)
{
    __shared__ double red[kPathWaves];
    const PathDesc P = descs[blockIdx.x];
    if (!P.beta0) return;
    const auto beta_g = gmem(P.beta);
    const auto xbar_g = gmem(P.xbar);
    const double ym = *gmem(P.ybar);
    for (int l = 0; l < P.L; ++l) {
        double acc = 0.0;
        for (int i = threadIdx.x; i < P.p; i += kPathThreads) acc += xbar_g[i] * beta_g[(size_t)l * P.p + i];
        acc = wave_sum(acc);
        if (threadIdx.x % kWave == 0) red[threadIdx.x / kWave] = acc;
        __syncthreads();
        if (threadIdx.x == 0) {
            double t = 0.0;
            for (int w = 0; w < kPathWaves; ++w) t += red[w];
            gmem(P.beta0)[l] = ym - t;
        }
        __syncthreads();
    }
}

int launch_intercepts(const PathDesc *d_desc, int count, hipStream_t s)
{
    if (count <= 0) return OEM_OK;
    hipLaunchKernelGGL(intercept_kernel, dim3(count), dim3(kPathThreads), 0, s, d_desc);
    OEM_HIP_CHECK(hipGetLastError());
    return OEM_OK;
}

// ---------------------------------------------------------------- CV error

// MSE_{k,l} = (yy_k - 2 beta^T b_k + beta^T G_k beta) / n_k from held-out
// sums; with an intercept b0 the residual is y - b0 - x^T beta, which adds
// n_k b0^2 - 2 b0 sum_k y + 2 b0 beta^T colsum_k.  One workgroup per (fold,
// penalty, lambda).  Only the nonzero coefficients enter: their indices and
// values are gathered into LDS (ascending), then beta^T G_k beta is the sum
// over pairs of them, each thread taking pairs along a row of G_k.
__global__ __launch_bounds__(kPathThreads) void cv_mse_kernel(
    const double *__restrict__ Gk, const double *__restrict__ bk, const double *__restrict__ yyk,
    const int64_t *__restrict__ nk, const double *__restrict__ csk, const double *__restrict__ ysk,
    const double *__restrict__ beta0_folds, int K, int p, int npen, int L,
    const double *__restrict__ beta_folds, double *__restrict__ mse)
{
    extern __shared__ double cv_sm[];
    double *val = cv_sm;                                        // [p] nonzero values
    int *idx = reinterpret_cast<int *>(val + p);                // [p] their indices
    __shared__ double red[3 * kPathWaves];
    __shared__ int wcnt[kPathWaves];
    const int t = threadIdx.x, lane = t % kWave, wave = t / kWave;
    const int l = blockIdx.x % L;
    const int pen = (blockIdx.x / L) % npen;
    const int k = blockIdx.x / (L * npen);
    const size_t path_l = ((size_t)k * npen + pen) * L + l;
    const double *beta = beta_folds + path_l * p;
    const double *G = Gk + (size_t)k * p * p;
    double quad = 0.0, lin = 0.0, mix = 0.0;
    // gather the nonzero coefficients in ascending order
    int nnz = 0;
    for (int base = 0; base < p; base += kPathThreads) {
        const int j = base + t;
        const double b = j < p ? beta[j] : 0.0;
        const bool nz = b != 0.0;
        const uint64_t ball = __ballot(nz);
        if (lane == 0) wcnt[wave] = __popcll(ball);
        __syncthreads();
        int before = 0, total = 0;
        for (int w = 0; w < kPathWaves; ++w) {
            before += w < wave ? wcnt[w] : 0;
            total += wcnt[w];
        }
        if (nz) {
            const int e = nnz + before + __popcll(ball & ((1ull << lane) - 1ull));
            val[e] = b;
            idx[e] = j;
            lin += b * bk[(size_t)k * p + j];
            if (beta0_folds) mix += b * csk[(size_t)k * p + j];
        }
        nnz += total;
        __syncthreads();
    }
    // beta^T G beta over the pairs (a, c) of nonzero coefficients
    const int pairs = nnz * nnz;
    for (int e = t; e < pairs; e += kPathThreads) {
        const int a = e / nnz, c = e - a * nnz;
        quad += val[a] * (G[(size_t)idx[a] * p + idx[c]] * val[c]);
    }
    quad = wave_sum(quad);
    lin = wave_sum(lin);
    mix = wave_sum(mix);
    if (lane == 0) {
        red[wave] = quad;
        red[kPathWaves + wave] = lin;
        red[2 * kPathWaves + wave] = mix;
    }
    __syncthreads();
    if (t == 0) {
        double q2 = 0.0, l2 = 0.0, m2 = 0.0;
        for (int w = 0; w < kPathWaves; ++w) {
            q2 += red[w];
            l2 += red[kPathWaves + w];
            m2 += red[2 * kPathWaves + w];
        }
        double sse = yyk[k] - 2.0 * l2 + q2;
        if (beta0_folds) {
            const double b0 = beta0_folds[path_l];
            sse += (double)nk[k] * b0 * b0 - 2.0 * b0 * ysk[k] + 2.0 * b0 * m2;
        }
        mse[((size_t)pen * K + k) * L + l] = sse / (double)nk[k];
    }
}

// cvm, cvsd per (penalty, lambda); i_min, i_1se per penalty; best penalty.
__global__ void cv_select_kernel(const double *__restrict__ mse, const int64_t *__restrict__ nk,
                                 int K, int npen, int L, double *__restrict__ cvm,
                                 double *__restrict__ cvsd, int32_t *__restrict__ i_min,
                                 int32_t *__restrict__ i_1se, int32_t *__restrict__ best)
{
    int64_t ntot = 0;
    for (int k = 0; k < K; ++k) ntot += nk[k];
    const double n = (double)ntot;
    for (int e = threadIdx.x; e < npen * L; e += blockDim.x) {
        const int pen = e / L, l = e % L;
        double m = 0.0;
        for (int k = 0; k < K; ++k) m += (double)nk[k] * mse[((size_t)pen * K + k) * L + l];
        m /= n;
        double v = 0.0;
        for (int k = 0; k < K; ++k) {
            const double dv = mse[((size_t)pen * K + k) * L + l] - m;
            v += (double)nk[k] * dv * dv;
        }
        cvm[e] = m;
        cvsd[e] = sqrt(v / (n * (K - 1)));
    }
    __syncthreads();
    for (int pen = threadIdx.x; pen < npen; pen += blockDim.x) {
        int im = 0;
        for (int l = 1; l < L; ++l)
            if (cvm[(size_t)pen * L + l] < cvm[(size_t)pen * L + im]) im = l;
        const double thr = cvm[(size_t)pen * L + im] + cvsd[(size_t)pen * L + im];
        int i1 = im;
        for (int l = 0; l < L; ++l)
            if (cvm[(size_t)pen * L + l] <= thr) { i1 = l; break; }
        if (i_min) i_min[pen] = im;
        if (i_1se) i_1se[pen] = i1;
    }
    __syncthreads();
    if (threadIdx.x == 0 && best) {
        int b = 0;
        double bv = INFINITY;
        for (int pen = 0; pen < npen; ++pen) {
            double mn = cvm[(size_t)pen * L];
            for (int l = 1; l < L; ++l) mn = fmin(mn, cvm[(size_t)pen * L + l]);
            if (mn < bv) { bv = mn; b = pen; }
        }
        *best = b;
    }
}

int launch_cv(const double *Gk, const double *bk, const double *yyk, const int64_t *nk,
              const double *csk, const double *ysk, const double *beta0_folds, int K,
              int p, int npen, int L, const double *beta_folds, double *mse, double *cvm,
              double *cvsd, int32_t *i_min, int32_t *i_1se, int32_t *best, hipStream_t s)
{
    const size_t lds = (size_t)p * (sizeof(double) + sizeof(int));
    OEM_HIP_CHECK(hipFuncSetAttribute((const void *)cv_mse_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                      (int)lds));
    hipLaunchKernelGGL(cv_mse_kernel, dim3(K * npen * L), dim3(kPathThreads), lds, s, Gk, bk, yyk, nk,
                       csk, ysk, beta0_folds, K, p, npen, L, beta_folds, mse);
    OEM_HIP_CHECK(hipGetLastError());
    hipLaunchKernelGGL(cv_select_kernel, dim3(1), dim3(256), 0, s, mse, nk, K, npen, L, cvm, cvsd,
                       i_min, i_1se, best);
    OEM_HIP_CHECK(hipGetLastError());
    return OEM_OK;
}

} // namespace oem
