// OEM path kernel on a working set of coordinates with exact screening of the
// others (Section 2.1 iteration, Section 2.2 updates).
//
// Every update of Section 2.1 leaves a coordinate j at zero exactly when its
// thresholding input is small: |u_j| <= w_j lambda (lasso, MCP, SCAD; times
// alpha for the elastic net) or ||u_g|| <= c_g lambda for a group.  For a
// coordinate that is zero, u_j = c_j - (G beta)_j.  Only the coordinates of
// the working set W below move, so between two iterates
//     |u_j(beta) - u_j(beta')| <= r_j max_k |beta_k - beta'_k|,
// r_j = sum_{k in W} |G_jk|  (for a group, sqrt(sum_{j in g} r_j^2) bounds the
// change of ||u_g||).  So after an exact evaluation of u at a reference beta,
// a zero coordinate with slack s_j = threshold - |u_j| stays zero in every
// update whose input beta is within s_j / r_j of the reference (max norm).
//
// The kernel keeps a working set W of at most C = 32 NW coordinates (whole
// groups for the group lasso): the nonzero coordinates and the zero ones
// closest to their threshold (smallest s_j).  G restricted to W lives
// in registers.  Wave w owns slots [32 w, 32 w + 32); lanes l and l + 32 both
// own slot 32 w + l and hold its row of G_WW, split by columns: lane l the
// first C / 2 columns, lane l + 32 the rest.  An update reads beta_W from LDS
// as broadcast loads, forms the two half-row products, joins them with one
// cross-half lane swap (both lanes then hold the same sum, and compute the
// same update), and writes the new beta of the slot back to LDS; with more
// than one wave that write is followed by the update's only barrier.  The
// stopping rule needs max |beta| (one reduction); whether every change is
// within tol times it, and whether any coordinate drifted past the screening
// bound, are wave ballots.  The coordinates outside W are not touched while
// the drift max_k |beta_k - beta_ref_k| stays below S = min over j outside W
// of s_j / r_j.  At a check point - the start of the path, and whenever the
// drift reaches S - the kernel forms G beta for all p coordinates from the
// columns of the nonzero coordinates (from LDS in the one-wave kernel, else
// from memory), which gives the exact u, the stationarity check, the
// objective and new keys, and rebuilds W when a coordinate outside it needs
// to enter.  The iterates are those of the full update: the coordinates
// outside W are exactly the ones the full update would leave at zero.  At
// the end of a lambda the outputs need G beta on W only (every coordinate
// outside W is zero and inside its threshold), and the slacks s_j of the
// next lambda follow from the reference's |u_j| with the smaller threshold:
// W and the reference carry on while the drift stays below the new S, and a
// check point is taken only when it does not.
//
// When more than C coordinates need W, the kernel stops before that lambda:
// *lstart receives the lambda index and bws the coefficients (standardised)
// of the lambda before it, and the next kernel of the launch plan continues
// from there with the same warm start.
#include <cfloat>

#include "path_common.h"

namespace oem {

constexpr int kWsCB = 32;   // slots per wave

static __host__ __device__ inline int ws_pow2(int v)
{
    int s = 2;
    while (s < v) s <<= 1;
    return s;
}

// G stays in LDS for the one-wave kernel (p <= 128)
constexpr int kWsLdsGMaxP = 128;

// LDS a working-set workgroup reserves (more than half of a CU's 160 KB)
constexpr size_t kWsReserveLds = 100 * 1024;

size_t path_ws_lds_bytes(int NW, int pcap)
{
    const int C = NW * kWsCB, PSC = ws_pow2(pcap);
    const size_t gl = NW == 1 ? (size_t)pcap * pcap : 0;
    const size_t dbl = 2 * (size_t)C + 8 * (size_t)NW + 4 * (size_t)NW + 6 * (size_t)pcap + 2 * (size_t)PSC + 2 * (size_t)C + gl;
    const size_t ints = (size_t)PSC + 2 * (size_t)pcap + 2 * (size_t)C + 2 * (size_t)C + 16 + 2 * (size_t)NW;
    return dbl * sizeof(double) + ints * sizeof(int) + 64;
}

// The path of one workgroup.  KIND >= 0: the penalty kind as a compile-time
// constant (the update and the penalty terms then carry no branches on it);
// KIND < 0: the kind is read from the descriptor.
template <int NW, int KIND>
__device__ __forceinline__ void path_ws_body(const PathDesc &P, int first, int pcap)
{
    constexpr int CB = kWsCB, C = NW * CB, HC = C / 2, NT = 64 * NW;
    const int p = P.p, L = P.L;
    const int kind = KIND >= 0 ? KIND : P.kind;
    const bool grp = (kind == OEM_GRP_LASSO);
    const int nkeys = grp ? P.ngroups : p;
    const int PS = ws_pow2(nkeys), PSC = ws_pow2(pcap);

    extern __shared__ double sm[];
    double *bsl = sm;                         // [2][C] beta of each slot (double-buffered)
    double *dm = bsl + 2 * C;                 // [2][NW][4] per-wave stopping-rule values
    double *fin = dm + 8 * NW;                // [4][NW] per-wave check-point sums
    double *bfull = fin + 4 * NW;             // [pcap] beta (zero outside W)
    double *gfull = bfull + pcap;             // [pcap] G beta
    double *r1 = gfull + pcap;                // [pcap] 1 / r of each key for the current W (r_j = sum_{k in W} |G_jk|; a group's sqrt(sum r_j^2))
    double *key = r1 + pcap;                  // [PSC] s_j / r_j, -1 when j needs W
    double *ab = key + PSC;                   // [C] values of the nonzero coordinates
    double *cl = ab + C;                      // [pcap] c
    double *scl = cl + pcap;                  // [pcap] column scales
    double *wl = scl + pcap;                  // [pcap] penalty weights; group lasso: c_g of each group
    double *usq = wl + pcap;                  // [NW][CB] u^2 of each wave's slots (group lasso)
    double *kref = usq + C;                   // [PSC] |u_j| (||u_g||) of each key at the reference beta
    double *gls = kref + PSC;                 // [pcap pcap] G (one-wave kernel only)
    int *kid = reinterpret_cast<int *>(gls + (NW == 1 ? pcap * pcap : 0));   // [PSC] coordinate (group) of each key
    // [2][C] per-slot changes of the updates (more than one wave): the keys'
    // area, which only a check point uses (PSC >= 2 C whenever NW > 1)
    double *dls = key;
    int *slot_of = kid + PSC;                 // [pcap] slot of each coordinate, -1 outside W
    int *gof = slot_of + pcap;                // [pcap] group of each coordinate
    int *ws = gof + pcap;                     // [C] coordinate of each slot, -1 when empty
    int *aj = ws + C;                         // [C] indices of the nonzero coordinates
    int *gl = aj + C;                         // [2 C] lane range of each slot's group in its wave
    int *misc = gl + 2 * C;                   // [16 + 2 NW] counters and flags

    const auto G = gmem(P.G);
    const auto lambda_g = gmem(P.lambda);
    const auto beta_g = gmem(P.beta);
    const auto beta_std_g = gmem(P.beta_std);
    const auto kkt_g = gmem(P.kkt);
    const auto obj_g = gmem(P.obj);
    const auto iters_g = gmem(P.iters);
    const auto c_g = gmem(P.c);
    const auto s_g = gmem(P.s);
    const auto w_g = gmem(P.w);
    const auto gstart = gmem(P.gstart);
    const auto gidx = gmem(P.gidx);
    const auto cgw = gmem(P.cg);
    const auto bws = gmem(P.bws);
    const int t = threadIdx.x, lane = t % kWave, wave = t / kWave;
    const int half = lane / CB;               // which half of the slot's row this lane holds
    const int os = CB * wave + lane % CB;     // slot owned by this lane (and by its partner lane)
    const double d = *P.d;
    const double yyn = *P.yyn;
    const double inv_d = 1.0 / d;
    const double thr_scale = (kind == OEM_ENET) ? P.alpha : 1.0;

    // Workgroup barrier.  A one-wave workgroup needs none: its LDS operations
    // complete in order, so a wavefront-scope fence (which also keeps global
    // stores from being waited for) is enough.
    auto sync = [&]() {
        if constexpr (NW == 1) {
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            __builtin_amdgcn_wave_barrier();
        } else {
            __syncthreads();
        }
    };
    // G from LDS (one wave) or from memory
    auto gat = [&](size_t idx) -> double {
        if constexpr (NW == 1)
            return gls[idx];
        else
            return G[idx];
    };

    int l0 = first ? 0 : *P.lstart;
    if (l0 >= L) return;

    for (int j = t; j < p; j += NT) {
        cl[j] = c_g[j];
        scl[j] = s_g[j];
        if (!grp) wl[j] = w_g ? w_g[j] : 1.0;
    }
    if (grp)
        for (int g = t; g < P.ngroups; g += NT) wl[g] = cgw[g];
    const double *cgl = wl;                   // group weights from LDS
    if constexpr (NW == 1) {
        const int pp = p * p;
        for (int e = t; e < pp; e += NT) gls[e] = G[e];
        sync();
    }
    // start coefficients, empty W (r1 is set when W is built)
    for (int j = t; j < p; j += NT) {
        r1[j] = 0.0;
        bfull[j] = l0 > 0 ? bws[j] : 0.0;
        slot_of[j] = -1;
    }
    for (int s = t; s < C; s += NT) {
        ws[s] = -1;
        gl[2 * s] = gl[2 * s + 1] = s % CB;
    }
    if (grp)
        for (int g = t; g < P.ngroups; g += NT)
            for (int q = gstart[g]; q < gstart[g + 1]; ++q) gof[gidx[q]] = g;
    sync();

    // per-slot state of the owning lanes (the same in both)
    double Gr[HC];                // row W(os) of G_WW, columns [half HC, half HC + HC)
#pragma unroll
    for (int c = 0; c < HC; ++c) Gr[c] = 0.0;
    int jc = -1;                  // coordinate of the owned slot
    double bt = 0.0, bref = 0.0, ct = 0.0, wt = 1.0;
    int gA = lane, gB = lane, gmaxw = 0;   // group lane range, largest group of the wave
    double S = -1.0;              // drift allowed before the next check point
    double Sthr = -1.0;           // S less a relative margin for rounding
    Upd q{};
    double lamc = 0.0;            // c_g lambda of the owned slot's group

    // (G_WW beta_W) of the owned slot: beta_W from bsl[buf] by broadcast
    // loads (each half reads its own column range), four accumulators, then
    // the two halves joined.  The join adds the same two values in the same
    // order in both lanes, so both get the same result.
    auto symv = [&](int buf) -> double {
        const double *bb = bsl + buf * C + half * HC;
        double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
        // the operand reads of a block of 16 columns are issued together
        // (one LDS latency per block rather than per pair of reads)
        constexpr int SB = HC < 32 ? HC : 32;
#pragma unroll
        for (int c0 = 0; c0 < HC; c0 += SB) {
            double2 vb[SB / 2];
#pragma unroll
            for (int u = 0; u < SB / 2; ++u) vb[u] = *reinterpret_cast<const double2 *>(bb + c0 + 2 * u);
#pragma unroll
            for (int u = 0; u < SB / 2; u += 2) {
                a0 += Gr[c0 + 2 * u] * vb[u].x;
                a1 += Gr[c0 + 2 * u + 1] * vb[u].y;
                a2 += Gr[c0 + 2 * u + 2] * vb[u + 1].x;
                a3 += Gr[c0 + 2 * u + 3] * vb[u + 1].y;
            }
        }
        const double sh = (a0 + a1) + (a2 + a3);
        const int lo = __double2loint(sh), hi = __double2hiint(sh);
        const auto pl = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
        const auto ph = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
        return __hiloint2double((int)ph[0], (int)pl[0]) + __hiloint2double((int)ph[1], (int)pl[1]);
    };
    // max over the 32 slots of the wave (lanes 0-31; lanes 32-63 hold the
    // same values), the same in every lane
    auto slot_max = [&](double v) -> double {
        v = fmax(v, dpp_mov<0xB1>(v));
        v = fmax(v, dpp_mov<0x4E>(v));
        v = fmax(v, dpp_mov<0x124>(v));
        v = fmax(v, dpp_mov<0x128>(v));
        return fmax(readlane_d(v, 0), readlane_d(v, 16));
    };
    auto set_upd = [&](double lam) {
        q = make_upd(kind, wt * lam, d, P.alpha, P.gamma);
        lamc = (grp && jc >= 0) ? cgl[gof[jc]] * lam : 0.0;
    };

    // The keys in W get kref = -inf: no bound for the next lambda comes
    // from them (after the check point's own writes of kref).
    auto mark_w = [&]() {
        for (int s = t; s < C; s += NT)
            if (ws[s] >= 0) kref[grp ? gof[ws[s]] : ws[s]] = -INFINITY;
    };

    // Check point at the current beta.  lam_end >= 0: the lambda whose
    // iterations just ended (outputs, stationarity, objective for index
    // l_end).  lam_next >= 0: the lambda the next updates use (screening
    // keys).  from_slots: beta is in the owners' registers (else in bfull).
    // keep: W is kept when every needed coordinate is in it and the drift
    // it then allows (the smallest key outside it) exceeds keep; otherwise
    // W is rebuilt (keep = inf always rebuilds).
    // Returns 1 when more than C coordinates need W (uniform).
    auto checkpoint = [&](int l_end, double lam_end, double lam_next, bool from_slots, double keep,
                          int it_end, bool conv_end) -> int {
        if (from_slots) {
            if (half == 0 && jc >= 0) bfull[jc] = bt;
            sync();
        }
        // nonzero coordinates in ascending order
        int nact = 0;
        for (int base = 0; base < p; base += NT) {
            const int j = base + t;
            const bool nz = j < p && bfull[j] != 0.0;
            const uint64_t ball = __ballot(nz);
            if (lane == 0) misc[16 + wave] = __popcll(ball);
            sync();
            int before = 0, total = 0;
#pragma unroll
            for (int w = 0; w < NW; ++w) {
                const int cw = misc[16 + w];
                before += (w < wave) ? cw : 0;
                total += cw;
            }
            if (nz) {
                const int k = nact + before + __popcll(ball & ((1ull << lane) - 1ull));
                if (k < C) {
                    aj[k] = j;
                    ab[k] = bfull[j];
                }
            }
            nact += total;
            sync();
        }
        if (nact > C) return 1;
        // G beta for every coordinate from the columns of the nonzero ones
        if constexpr (NW <= 2) {
            // rows in chunks of JM NT (one chunk for the one-wave kernel); the
            // indices and values of the nonzero coordinates are read once per
            // 16 columns, and each thread keeps 16 JM loads of G in flight
            constexpr int JM = NW == 1 ? (kWsLdsGMaxP + NT - 1) / NT : 4;
            for (int j0 = 0; j0 < p; j0 += JM * NT) {
                double acc[JM];
#pragma unroll
                for (int jj = 0; jj < JM; ++jj) acc[jj] = 0.0;
                for (int e0 = 0; e0 < nact; e0 += 16) {
                    int je[16];
                    double be[16];
#pragma unroll
                    for (int u = 0; u < 16; ++u) {
                        const int e = min(e0 + u, nact - 1);
                        be[u] = (e0 + u < nact) ? ab[e] : 0.0;
                        je[u] = aj[e];
                    }
#pragma unroll
                    for (int jj = 0; jj < JM; ++jj) {
                        if (j0 + jj * NT >= p) break;
                        const int j = min(j0 + t + jj * NT, p - 1);
                        double gv[16];
#pragma unroll
                        for (int u = 0; u < 16; ++u) gv[u] = gat((size_t)je[u] * p + j);
                        double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
#pragma unroll
                        for (int u = 0; u < 16; u += 4) {
                            a0 += gv[u] * be[u];
                            a1 += gv[u + 1] * be[u + 1];
                            a2 += gv[u + 2] * be[u + 2];
                            a3 += gv[u + 3] * be[u + 3];
                        }
                        acc[jj] += (a0 + a1) + (a2 + a3);
                    }
                }
#pragma unroll
                for (int jj = 0; jj < JM; ++jj)
                    if (j0 + t + jj * NT < p) gfull[j0 + t + jj * NT] = acc[jj];
            }
        } else {
            for (int j = t; j < p; j += NT) {
                double a[4] = {0.0, 0.0, 0.0, 0.0};
                for (int e0 = 0; e0 < nact; e0 += 16) {
                    double gv[16], bv[16];
#pragma unroll
                    for (int u = 0; u < 16; ++u) {
                        const int e = min(e0 + u, nact - 1);
                        bv[u] = (e0 + u < nact) ? ab[e] : 0.0;
                        gv[u] = gat((size_t)aj[e] * p + j);
                    }
#pragma unroll
                    for (int u = 0; u < 16; ++u) a[u % 4] += gv[u] * bv[u];
                }
                gfull[j] = (a[0] + a[1]) + (a[2] + a[3]);
            }
        }
        sync();
        // exact u, outputs of the finished lambda, screening keys of the next
        const bool has_next = lam_next >= 0.0;
        double kv = 0.0, penv = 0.0, quad = 0.0, lin = 0.0, smin = INFINITY;
        int nneed = 0;
        if (!grp) {
            for (int j = t; j < p; j += NT) {
                const double b = bfull[j], g = gfull[j], cj = cl[j];
                const double wj = wl[j];
                if (lam_end >= 0.0) {
                    const double lw = wj * lam_end;
                    const double gr = g - cj;
                    if (b == 0.0)
                        kv = nmax(kv, pos(fabs(gr) - thr_scale * lw));
                    else
                        kv = nmax(kv, fabs(gr + sgn(b) * pen_deriv(kind, fabs(b), lw, P.alpha, P.gamma)));
                    penv += pen_value(kind, b, lw, P.alpha, P.gamma);
                    quad += b * g;
                    lin += cj * b;
                    beta_g[(size_t)l_end * p + j] = b / scl[j];
                    if (beta_std_g) beta_std_g[(size_t)l_end * p + j] = b;
                    bws[j] = b;
                }
                if (has_next) {
                    const double u = cj + (d * b - g);
                    const double thr = wj * lam_next * thr_scale;
                    const double sl = thr - fabs(u);
                    const bool need = (b != 0.0) || !(sl > 1e-12 * thr);
                    key[j] = need ? -1.0 : sl;
                    kref[j] = fabs(u);
                    kid[j] = j;
                    nneed += need ? 1 : 0;
                    if (slot_of[j] < 0) smin = fmin(smin, need ? -1.0 : fmin(sl * r1[j], DBL_MAX));
                }
            }
        } else {
            for (int g = t; g < P.ngroups; g += NT) {
                const int q0 = gstart[g], q1 = gstart[g + 1];
                double uu = 0.0, bb = 0.0, gg = 0.0;
                bool nz = false;
                for (int qq = q0; qq < q1; ++qq) {
                    const int j = gidx[qq];
                    const double b = bfull[j], gv = gfull[j], cj = cl[j];
                    const double u = cj + (d * b - gv);
                    uu += u * u;
                    bb += b * b;
                    gg += (gv - cj) * (gv - cj);
                    nz |= b != 0.0;
                    if (lam_end >= 0.0) {
                        quad += b * gv;
                        lin += cj * b;
                        beta_g[(size_t)l_end * p + j] = b / scl[j];
                        if (beta_std_g) beta_std_g[(size_t)l_end * p + j] = b;
                        bws[j] = b;
                    }
                }
                if (lam_end >= 0.0) {
                    const double lc = lam_end * cgl[g];
                    const double bn = sqrt(bb);
                    double v;
                    if (bn > 0.0) {
                        double ss = 0.0;
                        for (int qq = q0; qq < q1; ++qq) {
                            const int j = gidx[qq];
                            const double e = (gfull[j] - cl[j]) + lc * bfull[j] / bn;
                            ss += e * e;
                        }
                        v = sqrt(ss);
                    } else {
                        v = pos(sqrt(gg) - lc);
                    }
                    kv = nmax(kv, v);
                    penv += lc * bn;
                }
                if (has_next) {
                    const double thr = cgl[g] * lam_next;
                    const double un = sqrt(uu);
                    const double sl = thr - un;
                    const bool need = nz || !(sl > 1e-12 * thr);
                    key[g] = need ? -1.0 : sl;
                    kref[g] = un;
                    kid[g] = g;
                    nneed += need ? (q1 - q0) : 0;
                    if (slot_of[gidx[q0]] < 0) smin = fmin(smin, need ? -1.0 : fmin(sl * r1[g], DBL_MAX));
                }
            }
        }
        if (has_next)
            for (int i = nkeys + t; i < PS; i += NT) {
                key[i] = INFINITY;
                kid[i] = -1;
            }
        // block reductions: max kv, sums penv quad lin, min smin, sum nneed
        if (lam_end >= 0.0) {   // the outputs of a finished lambda only
            kv = wave_max(kv);
            penv = wave_sum(penv);
            quad = wave_sum(quad);
            lin = wave_sum(lin);
        }
        smin = -wave_max(-smin);
        const double nn = wave_sum((double)nneed);
        if (lane == 0) {
            fin[0 * NW + wave] = kv;
            fin[1 * NW + wave] = penv;
            fin[2 * NW + wave] = quad;
            fin[3 * NW + wave] = lin;
            dm[wave * 4 + 0] = smin;      // dm[0][*] is free between updates
            dm[wave * 4 + 1] = nn;
        }
        sync();
        double SM = dm[0], NN = dm[1];
        for (int w = 1; w < NW; ++w) {
            SM = fmin(SM, dm[w * 4]);
            NN += dm[w * 4 + 1];
        }
        if (lam_end >= 0.0 && t == 0) {
            double K = fin[0], Pn = fin[NW], Q = fin[2 * NW], Li = fin[3 * NW];
            for (int w = 1; w < NW; ++w) {
                K = fmax(K, fin[w]);
                Pn += fin[NW + w];
                Q += fin[2 * NW + w];
                Li += fin[3 * NW + w];
            }
            if (kkt_g) kkt_g[l_end] = K;
            if (obj_g) obj_g[l_end] = 0.5 * Q - Li + 0.5 * yyn + Pn;
            if (iters_g) iters_g[l_end] = conv_end ? it_end : -it_end;
        }
        if (!has_next) return 0;
        if (NN > (double)C) return 1;
        if (SM > 0.0 && SM > keep) {    // every needed coordinate is in W
            S = SM;
            Sthr = S * (1.0 - 1e-9);
            bref = bt;
            mark_w();
            sync();            // dm and fin are read before they are reused
            return 0;
        }
        // rebuild W: order the keys ascending, needed ones first
        if constexpr (NW == 1) {
            // At most 128 keys, two per lane.  Each key gets a 64-bit order
            // code: its bit pattern (keys are -1 for needed coordinates, else
            // positive, +inf for padding) with the low 8 bits replaced by its
            // position, so codes are distinct and ordered as the keys up to
            // 2^-44 relative.  A key's rank among the codes is its place.
            sync();
            double mk[2];
            int mi[2], rk[2] = {0, 0};
            unsigned long long mc[2];
#pragma unroll
            for (int e = 0; e < 2; ++e) {
                const int i = t + 64 * e;
                mk[e] = i < PS ? key[i] : INFINITY;
                mi[e] = i < PS ? kid[i] : -1;
                const unsigned long long kb = (unsigned long long)__double_as_longlong(mk[e]);
                mc[e] = mk[e] < 0.0 ? (unsigned long long)i : (((kb < 256ull ? 256ull : kb) & ~255ull) | (unsigned long long)i);
            }
            sync();
            unsigned long long *code = reinterpret_cast<unsigned long long *>(key);
#pragma unroll
            for (int e = 0; e < 2; ++e)
                if (t + 64 * e < PS) code[t + 64 * e] = mc[e];
            sync();
            for (int j0 = 0; j0 < PS; j0 += 8) {
                unsigned long long cc[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) cc[u] = code[min(j0 + u, PS - 1)];
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const int jv = j0 + u < PS;
#pragma unroll
                    for (int e = 0; e < 2; ++e) rk[e] += jv & (int)(cc[u] < mc[e]);
                }
            }
            sync();
#pragma unroll
            for (int e = 0; e < 2; ++e)
                if (t + 64 * e < PS) {
                    key[rk[e]] = mk[e];
                    kid[rk[e]] = mi[e];
                }
        } else {
            // bitonic sort
            for (int k = 2; k <= PS; k <<= 1)
                for (int jj = k >> 1; jj > 0; jj >>= 1) {
                    sync();
                    for (int i = t; i < PS; i += NT) {
                        const int ixj = i ^ jj;
                        if (ixj > i) {
                            // compare-exchange with selects (stores are unconditional)
                            const bool up = (i & k) == 0;
                            const double a = key[i], b = key[ixj];
                            const int ta = kid[i], tb = kid[ixj];
                            const bool sw = (a > b) == up;
                            key[i] = sw ? b : a;
                            key[ixj] = sw ? a : b;
                            kid[i] = sw ? tb : ta;
                            kid[ixj] = sw ? ta : tb;
                        }
                    }
                }
        }
        sync();
        for (int s = t; s < C; s += NT)
            if (ws[s] >= 0) slot_of[ws[s]] = -1;
        sync();
        if (!grp) {
            for (int s = t; s < C; s += NT) ws[s] = (s < nkeys) ? kid[s] : -1;
            if (t == 0) misc[0] = 0;
        } else if (t == 0) {
            // whole groups into waves, first fit, in key order; stop at the
            // first group that does not fit
            for (int s = 0; s < C; ++s) {
                ws[s] = -1;
                gl[2 * s] = gl[2 * s + 1] = s % CB;
            }
            int fill[NW];
            for (int w = 0; w < NW; ++w) fill[w] = 0;
            int ovf = 0;
            for (int i = 0; i < nkeys; ++i) {
                const int g = kid[i];
                if (g < 0) break;   // padding: every group has been placed
                const int q0 = gstart[g], sz = gstart[g + 1] - q0;
                int w = 0;
                while (w < NW && fill[w] + sz > CB) ++w;
                if (w == NW) {
                    if (key[i] < 0.0) ovf = 1;
                    break;
                }
                for (int m = 0; m < sz; ++m) {
                    const int s = CB * w + fill[w] + m;
                    ws[s] = gidx[q0 + m];
                    gl[2 * s] = fill[w];
                    gl[2 * s + 1] = fill[w] + sz;
                }
                fill[w] += sz;
            }
            misc[0] = ovf;
        }
        sync();
        if (misc[0]) return 1;
        for (int s = t; s < C; s += NT)
            if (ws[s] >= 0) slot_of[ws[s]] = s;
        // The drift bound of the new W.  Only coordinates in W move, so
        // r_j = sum_{k in W} |G_jk| bounds |u_j(beta) - u_j(beta')| per unit
        // of max_k |beta_k - beta'_k| (rows of G for the W coordinates,
        // coalesced over j; gfull is free here).  S is the smallest s_k / r_k
        // outside W.
        for (int j0 = 0; j0 < p; j0 += NT) {
            const int j = min(j0 + t, p - 1);
            double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
            for (int s0 = 0; s0 < C; s0 += 16) {
                double gv[16];
#pragma unroll
                for (int u = 0; u < 16; ++u) {
                    const int jk = ws[s0 + u];
                    gv[u] = jk >= 0 ? fabs(gat((size_t)jk * p + j)) : 0.0;
                }
#pragma unroll
                for (int u = 0; u < 16; u += 4) {
                    a0 += gv[u];
                    a1 += gv[u + 1];
                    a2 += gv[u + 2];
                    a3 += gv[u + 3];
                }
            }
            if (j0 + t < p) gfull[j0 + t] = (a0 + a1) + (a2 + a3);
        }
        sync();
        double sb = INFINITY;
        if (!grp) {
            for (int j = t; j < p; j += NT) {
                const double rinv = 1.0 / gfull[j];
                r1[j] = rinv;
                if (slot_of[j] < 0)
                    sb = fmin(sb, fmin((wl[j] * lam_next * thr_scale - kref[j]) * rinv, DBL_MAX));
            }
        } else {
            for (int g = t; g < P.ngroups; g += NT) {
                const int q0 = gstart[g], q1 = gstart[g + 1];
                double rr = 0.0;
                for (int qq = q0; qq < q1; ++qq) rr += gfull[gidx[qq]] * gfull[gidx[qq]];
                const double rinv = 1.0 / sqrt(rr);
                r1[g] = rinv;
                if (slot_of[gidx[q0]] < 0) sb = fmin(sb, fmin((cgl[g] * lam_next - kref[g]) * rinv, DBL_MAX));
            }
        }
        sb = -wave_max(-sb);
        if (lane == 0) dm[wave * 4 + 3] = sb;
        sync();
        S = dm[3];
        for (int w = 1; w < NW; ++w) S = fmin(S, dm[w * 4 + 3]);
        Sthr = S * (1.0 - 1e-9);
        mark_w();
        // both lanes of a slot take its new coordinate; G_WW into registers
        jc = ws[os];
        bt = jc >= 0 ? bfull[jc] : 0.0;
        bref = bt;
        ct = jc >= 0 ? cl[jc] : 0.0;
        wt = jc >= 0 ? wl[jc] : 1.0;
        if (grp) {
            gA = gl[2 * os];
            gB = gl[2 * os + 1];
            int m = 0;
            for (int c = 0; c < CB; ++c) m = max(m, gl[2 * (CB * wave + c) + 1] - gl[2 * (CB * wave + c)]);
            gmaxw = m;
        }
#pragma unroll
        for (int c = 0; c < HC; ++c) {
            const int jcol = ws[half * HC + c];
            Gr[c] = (jcol >= 0 && jc >= 0) ? gat((size_t)jcol * p + jc) : 0.0;
        }
        set_upd(lam_next);
        sync();
        return 0;
    };

    // End of a lambda without forming G beta over all p.  It applies when the
    // final beta is within the screening bound of the reference (no drift):
    // then every coordinate outside W is zero with |u_j| below its threshold,
    // so its stationarity violation is exactly zero, and the outputs need
    // G beta on W only, which is gfin (the updates' last product G_WW beta_W,
    // beta being zero outside W).  The bound for the next lambda comes from
    // the reference's |u_j| (||u_g||) and the new thresholds.  Returns 0 when
    // W, the reference and the new bound carry on to the next lambda, 2 when
    // the outputs are written but the next lambda needs a check point first.
    auto light_end = [&](int l_end, double lam_end, double lam_next, double gfin, int it_end,
                         bool conv_end) -> int {
        if (half == 0 && jc >= 0) {
            bfull[jc] = bt;
            gfull[jc] = gfin;
        }
        const double Dw = slot_max(jc >= 0 ? fabs(bt - bref) : 0.0);
        sync();
        const bool has_next = lam_next >= 0.0;
        double kv = 0.0, penv = 0.0, quad = 0.0, lin = 0.0, smin = INFINITY;
        int nneed = 0;
        if (!grp) {
            for (int j = t; j < p; j += NT) {
                const size_t o = (size_t)l_end * p + j;
                if (slot_of[j] >= 0) {
                    const double b = bfull[j], g = gfull[j], cj = cl[j];
                    const double lw = wl[j] * lam_end;
                    const double gr = g - cj;
                    if (b == 0.0)
                        kv = nmax(kv, pos(fabs(gr) - thr_scale * lw));
                    else
                        kv = nmax(kv, fabs(gr + sgn(b) * pen_deriv(kind, fabs(b), lw, P.alpha, P.gamma)));
                    penv += pen_value(kind, b, lw, P.alpha, P.gamma);
                    quad += b * g;
                    lin += cj * b;
                    beta_g[o] = b / scl[j];
                    if (beta_std_g) beta_std_g[o] = b;
                    bws[j] = b;
                } else {
                    beta_g[o] = 0.0;
                    if (beta_std_g) beta_std_g[o] = 0.0;
                    bws[j] = 0.0;
                    if (has_next) {
                        const double thr = wl[j] * lam_next * thr_scale;
                        const double sl = thr - kref[j];
                        nneed += (sl > 1e-12 * thr) ? 0 : 1;
                        smin = fmin(smin, fmin(sl * r1[j], DBL_MAX));
                    }
                }
            }
        } else {
            // coordinates outside W: zero outputs
            for (int j = t; j < p; j += NT)
                if (slot_of[j] < 0) {
                    const size_t o = (size_t)l_end * p + j;
                    beta_g[o] = 0.0;
                    if (beta_std_g) beta_std_g[o] = 0.0;
                    bws[j] = 0.0;
                }
            // groups in W (whole groups, members in member order on
            // consecutive slots): the first slot of each takes its sums
            for (int s2 = t; s2 < C; s2 += NT) {
                const int j0 = ws[s2], l2 = s2 % CB, sb = s2 - l2;
                if (j0 < 0 || gl[2 * s2] != l2) continue;
                const int m1 = gl[2 * s2 + 1];
                double bb = 0.0, gg = 0.0;
                for (int m = l2; m < m1; ++m) {
                    const int j = ws[sb + m];
                    const double b = bfull[j], gv = gfull[j], cj = cl[j];
                    bb += b * b;
                    gg += (gv - cj) * (gv - cj);
                    quad += b * gv;
                    lin += cj * b;
                    beta_g[(size_t)l_end * p + j] = b / scl[j];
                    if (beta_std_g) beta_std_g[(size_t)l_end * p + j] = b;
                    bws[j] = b;
                }
                const double lc = lam_end * cgl[gof[j0]];
                const double bn = sqrt(bb);
                double v;
                if (bn > 0.0) {
                    double ss = 0.0;
                    for (int m = l2; m < m1; ++m) {
                        const int j = ws[sb + m];
                        const double e = (gfull[j] - cl[j]) + lc * bfull[j] / bn;
                        ss += e * e;
                    }
                    v = sqrt(ss);
                } else {
                    v = pos(sqrt(gg) - lc);
                }
                kv = nmax(kv, v);
                penv += lc * bn;
            }
            // groups outside W (kref = -inf in W): the next lambda's bound
            if (has_next)
                for (int g = t; g < P.ngroups; g += NT) {
                    const double thr = cgl[g] * lam_next;
                    const double sl = thr - kref[g];
                    nneed += (sl > 1e-12 * thr) ? 0 : 1;
                    smin = fmin(smin, fmin(sl * r1[g], DBL_MAX));
                }
        }
        kv = wave_max(kv);
        penv = wave_sum(penv);
        quad = wave_sum(quad);
        lin = wave_sum(lin);
        smin = -wave_max(-smin);
        const double nn = wave_sum((double)nneed);
        if (lane == 0) {
            fin[0 * NW + wave] = kv;
            fin[1 * NW + wave] = penv;
            fin[2 * NW + wave] = quad;
            fin[3 * NW + wave] = lin;
            dm[wave * 4 + 0] = smin;      // dm[0][*] is free between updates
            dm[wave * 4 + 1] = nn;
            dm[wave * 4 + 2] = Dw;
        }
        sync();
        double SM = dm[0], NN = dm[1], D = dm[2];
        for (int w = 1; w < NW; ++w) {
            SM = fmin(SM, dm[w * 4]);
            NN += dm[w * 4 + 1];
            D = fmax(D, dm[w * 4 + 2]);
        }
        if (t == 0) {
            double K = fin[0], Pn = fin[NW], Q = fin[2 * NW], Li = fin[3 * NW];
            for (int w = 1; w < NW; ++w) {
                K = fmax(K, fin[w]);
                Pn += fin[NW + w];
                Q += fin[2 * NW + w];
                Li += fin[3 * NW + w];
            }
            if (kkt_g) kkt_g[l_end] = K;
            if (obj_g) obj_g[l_end] = 0.5 * Q - Li + 0.5 * yyn + Pn;
            if (iters_g) iters_g[l_end] = conv_end ? it_end : -it_end;
        }
        int rc = 0;
        if (has_next) {
            const double St = SM * (1.0 - 1e-9);
            if (NN == 0.0 && SM > 0.0 && D < St) {
                S = SM;
                Sthr = St;
            } else {
                rc = 2;
            }
        }
        sync();            // dm and fin are read before they are reused
        return rc;
    };

    int cur = 0;
    if (checkpoint(-1, -1.0, lambda_g[l0], false, INFINITY, 0, false)) {
        if (t == 0) *P.lstart = l0;
        return;
    }
    bsl[cur * C + os] = bt;       // both lanes of a slot write the same value
    sync();
    double gb = symv(cur);

    double lam_cur = lambda_g[l0];
    for (int l = l0; l < L; ++l) {
        const double lam = lam_cur;
        const double lnext = (l + 1 < L) ? lambda_g[l + 1] : -1.0;   // in flight during the updates
        set_upd(lam);
        int it = 0;
        bool conv = false, drift = false;
        do {
            const double u = ct + (d * bt - gb);
            double bn;
            if (grp) {
                // the slot's group lies in lanes [gA, gB) of the first half;
                // u^2 of the wave's slots goes through LDS and each lane reads
                // its group's entries with independent reads (LDS operations
                // of one wave complete in order, so no barrier)
                double *uq = usq + wave * CB;
                if (half == 0) uq[lane] = u * u;
                double ss = 0.0;
                // the sum in member order (the order of the lambda_max
                // test); entries past the group are added as 0.0, which
                // leaves the sum unchanged and keeps the selects off the
                // chain of dependent additions
                if (gmaxw <= 16) {
                    // groups of up to 16: one batch of reads
                    double qv[16];
#pragma unroll
                    for (int k = 0; k < 16; ++k) qv[k] = uq[min(gA + k, CB - 1)];
#pragma unroll
                    for (int k = 0; k < 8; ++k) ss += (gA + k < gB) ? qv[k] : 0.0;
                    if (gmaxw > 8) {
#pragma unroll
                        for (int k = 8; k < 12; ++k) ss += (gA + k < gB) ? qv[k] : 0.0;
                    }
                    if (gmaxw > 12) {
#pragma unroll
                        for (int k = 12; k < 16; ++k) ss += (gA + k < gB) ? qv[k] : 0.0;
                    }
                } else {
                    for (int k0 = 0; k0 < gmaxw; k0 += 8) {
                        double qv[8];
#pragma unroll
                        for (int k = 0; k < 8; ++k) qv[k] = uq[min(gA + k0 + k, CB - 1)];
#pragma unroll
                        for (int k = 0; k < 8; ++k) ss += (gA + k0 + k < gB) ? qv[k] : 0.0;
                    }
                }
                // f = 1 - c_g lambda / ||u_g|| from 1 / ||u_g|| (the hardware
                // estimate and two Newton steps), which is within a few
                // units of 1e-16 of the quotient; where f is that close to
                // zero (or not finite), the exact quotient decides, as in the
                // lambda_max test
                double f = 0.0;
                if (ss > 0.0) {
                    double y = __builtin_amdgcn_rsq(ss);
                    const double h0 = 0.5 * y, e0 = fma(-(ss * y), y, 1.0);
                    y = fma(h0, e0, y);
                    const double h1 = 0.5 * y, e1 = fma(-(ss * y), y, 1.0);
                    y = fma(h1, e1, y);
                    f = fma(-lamc, y, 1.0);
                    if (!(fabs(f) >= 1e-12)) f = 1.0 - lamc / sqrt(ss);
                }
                bn = (jc >= 0 && f > 0.0) ? (u * inv_d) * f : 0.0;
            } else {
                bn = jc >= 0 ? update_fast(kind, u, q, P.gamma) : 0.0;
            }
            const double dl = fabs(bn - bt), mx = fabs(bn), dr = fabs(bn - bref);
            bt = bn;
            ++it;
            const int nxt = cur ^ 1;
            bsl[nxt * C + os] = bn;
            if (NW == 1) {
                sync();
                // the next product does not depend on the stopping test, so
                // its loads and products overlap the reduction below
                gb = symv(nxt);
                // stop when every change is within tol max|beta| (a NaN
                // change never is); drift when any coordinate moved S or more
                const double lim = P.tol * slot_max(mx);
                conv = __ballot(!(dl <= lim)) == 0;
                drift = __ballot(!(dr < Sthr)) != 0;
            } else {
                // each slot's change goes to LDS beside its new beta, with the
                // sign bit set when the slot drifted past the bound (a NaN
                // change counts as infinite, a NaN drift as drifted).  After
                // the barrier every wave forms max change, max |beta| and
                // the drift flag over all C slots itself (the same values in
                // the same lanes, so every wave takes the same decision),
                // beside the next product's operand reads and products
                const double dlc = dl <= INFINITY ? dl : INFINITY;
                dls[nxt * C + os] = (dr < Sthr) ? dlc : -dlc;
                sync();
                gb = symv(nxt);
                double DLv = 0.0, MXv = 0.0;
                bool drv = false;
#pragma unroll
                for (int s2 = lane; s2 < C; s2 += kWave) {
                    const double v = dls[nxt * C + s2];
                    DLv = fmax(DLv, fabs(v));
                    MXv = fmax(MXv, fabs(bsl[nxt * C + s2]));
                    drv |= signbit(v);
                }
                const double DL = wave_max(DLv), MX = wave_max(MXv);
                conv = DL <= P.tol * MX;
                drift = __ballot(drv) != 0;
            }
            cur = nxt;
            if (!conv && it < P.maxit && drift) {
                // the drift reached S: exact u again, new keys and bound; W
                // is rebuilt only when a coordinate outside it needs to enter
                // (rebuilding every time costs more than the extra check
                // points it saves)
                sync();   // dm[cur] is read before the check point reuses dm
                if (checkpoint(-1, -1.0, lam, true, 0.0, 0, false)) {
                    if (t == 0) *P.lstart = l;
                    return;
                }
                bsl[cur * C + os] = bt;
                sync();
                gb = symv(cur);
            }
        } while (!conv && it < P.maxit);
        sync();           // dm[cur] is read before the check point reuses dm
        // the final beta within the bound: outputs from W alone, and the
        // next lambda keeps W and the reference when the new bound allows
        const int le = drift ? 1 : light_end(l, lam, lnext, gb, it, conv);
        if (le != 0) {
            const int ov = le == 1 ? checkpoint(l, lam, lnext, true, 0.0, it, conv)
                                   : checkpoint(-1, -1.0, lnext, false, 0.0, 0, false);
            if (ov) {
                if (t == 0) *P.lstart = l + 1;
                return;
            }
            if (l + 1 < L) {
                // W may have been rebuilt: beta of the (new) slots
                bsl[cur * C + os] = bt;
                sync();
                gb = symv(cur);
            }
        }
        lam_cur = lnext;
    }
    if (t == 0) *P.lstart = L;
}

template <int NW>
__global__ __launch_bounds__(64 * NW) void path_ws_kernel(const PathDesc *__restrict__ descs,
                                                          const int *__restrict__ order, int first,
                                                          int pcap)
{
    const PathDesc P = descs[order[blockIdx.x]];
    if constexpr (NW == 1) {
        // one copy of the path per penalty kind (measured faster here; the
        // larger kernels keep one copy, which holds their register use down)
        switch (P.kind) {
        case OEM_LASSO: path_ws_body<NW, OEM_LASSO>(P, first, pcap); break;
        case OEM_ENET: path_ws_body<NW, OEM_ENET>(P, first, pcap); break;
        case OEM_MCP: path_ws_body<NW, OEM_MCP>(P, first, pcap); break;
        case OEM_SCAD: path_ws_body<NW, OEM_SCAD>(P, first, pcap); break;
        case OEM_GRP_LASSO: path_ws_body<NW, OEM_GRP_LASSO>(P, first, pcap); break;
        default: break;
        }
    } else {
        path_ws_body<NW, -1>(P, first, pcap);
    }
}

int launch_paths_ws(const PathDesc *d_desc, const int *d_order, int count, int nw, int first, int pmax,
                    hipStream_t s)
{
    if (count == 0) return OEM_OK;
    const void *kern;
    if (nw == 1)
        kern = (const void *)path_ws_kernel<1>;
    else if (nw == 2)
        kern = (const void *)path_ws_kernel<2>;
    else if (nw == 4)
        kern = (const void *)path_ws_kernel<4>;
    else
        return fail(OEM_E_INVAL, "working-set path kernel: 1, 2 or 4 waves");
    if (pmax > 2048) return fail(OEM_E_INVAL, "working-set path kernel needs p <= 2048");
    if (nw == 1 && pmax > kWsLdsGMaxP) return fail(OEM_E_INVAL, "one-wave working-set kernel needs p <= 128");
    // the per-slot changes of the updates share the keys' area
    if (nw > 1 && ws_pow2(pmax) < 2 * nw * kWsCB)
        return fail(OEM_E_INVAL, "working-set kernel of " + std::to_string(nw) + " waves needs p > " +
                                     std::to_string(nw * kWsCB));
    int pcap = pmax;
    // A path is a chain of dependent updates on one CU.  When the launch has
    // no more paths than the GPU has CUs, each workgroup asks for at least
    // kWsReserveLds of LDS, so that workgroups of other kernels running at the
    // same time (the next problem's Gram pass) are not placed beside it, where
    // they would compete for the LDS and issue slots its chain waits on.
    int dev = 0, ncu = 0;
    OEM_HIP_CHECK(hipGetDevice(&dev));
    OEM_HIP_CHECK(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    const size_t need = path_ws_lds_bytes(nw, pcap);
    const size_t lds = count <= ncu ? std::max(need, kWsReserveLds) : need;
    OEM_HIP_CHECK(hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    void *args[] = {(void *)&d_desc, (void *)&d_order, (void *)&first, (void *)&pcap};
    OEM_HIP_CHECK(hipLaunchKernel(kern, dim3(count), dim3(64 * nw), args, lds, s));
    return OEM_OK;
}

} // namespace oem
