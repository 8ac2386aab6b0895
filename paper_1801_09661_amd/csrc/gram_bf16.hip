// Streaming Gram pass on the BF16 matrix cores (mixed precision).
//
// Each FP32 value is split as x = hi + lo with hi = bf16(x) and
// lo = bf16(x - hi) (both round to nearest even).  The product x_i x_j is
// formed as hi_i hi_j + hi_i lo_j + lo_i hi_j on v_mfma_f32_32x32x16_bf16
// with FP32 accumulation; the dropped lo_i lo_j term is ~2^-16 relative and
// zero-mean off the diagonal.  On the diagonal it is not zero-mean, so the
// diagonal, X^T y and y^T y are accumulated in FP64 on the vector units from
// the loaded values.  Single BF16 (hi only, one product) is the reported
// variant.
//
// A workgroup owns one (fold, row split, super-block pair) of 32x32 tiles
// (super-blocks of up to 4 tiles = 128 columns) and streams its rows in
// chunks of 64:
//   load   thread (lane column l, row group rg) loads columns l, l+32, l+64,
//          l+96 of 8 rows (coalesced 128-byte row segments); the next
//          chunk's loads are issued before the current chunk's MFMAs;
//   stage  the thread splits its values and writes each column's 8 rows as
//          one 16-byte LDS store (consecutive lanes, consecutive columns:
//          no bank conflicts), so the panel is column-major in LDS and one
//          16-byte read is an MFMA operand (8 consecutive rows of a column);
//   mma    the waves form 2 pair groups x 2 k-groups: a pair group covers half
//          of the tile pairs, a k-group every other 16-row k-step, so each
//          wave reads a tile's operands once per k-step for several pairs;
//          the two k-groups' FP32 accumulators are added through LDS, in
//          wave order, when the workgroup finishes.  Diagonal and
//          off-diagonal super-block pairs are separate kernel launches.
// Partial tiles are FP32 and are summed over row splits in FP64 in a fixed
// order (deterministic, no floating-point atomics).
#include "gram_common.h"

namespace oem {

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x16_t __attribute__((ext_vector_type(16)));

constexpr int kBThreads = 256;
constexpr int kBWaves = kBThreads / kWave;
constexpr int kBTile = 32;                 // MFMA output tile
constexpr int kBMaxW = 4;                  // tiles per super-block side
constexpr int kBPanel = kBTile * kBMaxW;   // 128 columns per panel
constexpr int kBRows = 64;                 // rows per chunk: 4 MFMA k-steps of 16
constexpr int kBPitch = kBRows + 8;        // bf16 per staged column (144 bytes)

// Diagonal super-block: the 10 pairs (a, b), a <= b < 4, in two groups of 5
// that together need few operand tiles: group 0 = (0,0) (0,1) (0,2) (0,3)
// (3,3), group 1 = (1,1) (1,2) (1,3) (2,2) (2,3).
__host__ __device__ constexpr int dg_a(int grp, int t)
{
    return grp == 0 ? (t < 4 ? 0 : 3) : (t < 3 ? 1 : 2);
}
__host__ __device__ constexpr int dg_b(int grp, int t)
{
    return grp == 0 ? (t < 4 ? t : 3) : (t < 3 ? t + 1 : t - 1);
}

template <bool SPLIT>
__device__ inline void stage_cols(const float (&x)[8][4], __bf16 *hi, __bf16 *lo, int l, int rg)
{
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        bf16x8_t h, lw;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const float v = x[e][j];
            const __bf16 hb = (__bf16)v;
            h[e] = hb;
            if (SPLIT) lw[e] = (__bf16)(v - (float)hb);
        }
        const int c = l + 32 * j;
        *reinterpret_cast<bf16x8_t *>(hi + c * kBPitch + 8 * rg) = h;
        if (SPLIT) *reinterpret_cast<bf16x8_t *>(lo + c * kBPitch + 8 * rg) = lw;
    }
}

template <bool SPLIT>
__device__ inline f32x16_t mfma3(f32x16_t acc, const bf16x8_t &ah, const bf16x8_t &al,
                                 const bf16x8_t &bh, const bf16x8_t &bl)
{
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bh, acc, 0, 0, 0);
    if (SPLIT) {
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bl, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, bh, acc, 0, 0, 0);
    }
    return acc;
}

template <bool SPLIT, bool DIAG>
__global__ __launch_bounds__(kBThreads) void gram_bf16_kernel(
    const float *__restrict__ X, int64_t n, int64_t ldx, const double *__restrict__ y, GramGeom g,
    RowSource rs, float *__restrict__ partial, double *__restrict__ pvec, double *__restrict__ pscal)
{
    constexpr int NSLOT = DIAG ? 5 : 8;
    constexpr bool diag = DIAG;
    extern __shared__ char smem_raw[];
    const int lane = threadIdx.x % kWave;
    const int wave = threadIdx.x / kWave;
    const int lc = threadIdx.x % 32, rg = threadIdx.x / 32;

    // diagonal launch: blocks (k, s, I); off-diagonal launch: (k, s, I < J)
    const int nq = DIAG ? g.nsb : g.npsb - g.nsb;
    const int L = xcd_logical(blockIdx.x, gridDim.x);
    const int qq = L % nq;
    const int rest = L / nq;
    const int s = rest % g.nsplit;
    const int k = rest / g.nsplit;
    int I = 0, J = 0;
    if (DIAG) {
        I = J = qq;
    } else {
        int t = qq;
        for (I = 0; I < g.nsb; ++I) {
            const int cnt = g.nsb - I - 1;
            if (t < cnt) { J = I + 1 + t; break; }
            t -= cnt;
        }
    }
    const bool first_block = DIAG && (qq == 0);
    const int Wi = min(g.W, g.T - I * g.W);
    const int Wj = min(g.W, g.T - J * g.W);

    const int panel_elems = kBPanel * kBPitch;
    __bf16 *hiA = reinterpret_cast<__bf16 *>(smem_raw);
    __bf16 *loA = hiA + panel_elems;
    __bf16 *hiB = diag ? hiA : loA + panel_elems;
    __bf16 *loB = diag ? loA : hiB + panel_elems;

    // waves 2 pg, 2 pg + 1 form pair group pg and split the k-steps in two
    const int pg = wave / 2;
    const int ks0 = wave % 2;

    f32x16_t acc[NSLOT];
#pragma unroll
    for (int t = 0; t < NSLOT; ++t)
#pragma unroll
        for (int e = 0; e < 16; ++e) acc[t][e] = 0.0f;

    int64_t first, count;
    const int32_t *list;
    rows_of(g, rs, n, k, s, first, count, list);
    const int nchunks = (int)((count + kBRows - 1) / kBRows);
    const int colA = I * g.W * kBTile + lc, colB = J * g.W * kBTile + lc;
    const bool want_yy = first_block && (lc == 0);
    double sd[4] = {0.0, 0.0, 0.0, 0.0}, sxy[4] = {0.0, 0.0, 0.0, 0.0}, syy = 0.0;

    float xa[8][4], xb[8][4];
    double yv[8];
    auto load_chunk = [&](int c) {
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int64_t i = (int64_t)c * kBRows + 8 * rg + e;
            const bool ok = i < count;
            const int64_t row = ok ? row_at(first, list, i) : 0;
            const float *xr = X + row * ldx;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                xa[e][j] = (ok && colA + 32 * j < g.p) ? xr[colA + 32 * j] : 0.0f;
                if (!diag) xb[e][j] = (ok && colB + 32 * j < g.p) ? xr[colB + 32 * j] : 0.0f;
            }
            if (diag) yv[e] = ok ? y[row] : 0.0;
        }
    };
    auto stage_chunk = [&]() {
        stage_cols<SPLIT>(xa, hiA, loA, lc, rg);
        if (!diag) stage_cols<SPLIT>(xb, hiB, loB, lc, rg);
        if (diag) {
#pragma unroll
            for (int e = 0; e < 8; ++e) {
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const double xd = (double)xa[e][j];
                    sd[j] += xd * xd;
                    sxy[j] += xd * yv[e];
                }
                if (want_yy) syy += yv[e] * yv[e];
            }
        }
    };
    auto operand = [&](const __bf16 *panel, int tile, int ks) -> bf16x8_t {
        return *reinterpret_cast<const bf16x8_t *>(panel + (tile * kBTile + (lane % 32)) * kBPitch +
                                                   ks * 16 + 8 * (lane / 32));
    };
    auto mma_chunk = [&]() {
        for (int ks = ks0; ks < kBRows / 16; ks += 2) {
            if (DIAG) {
                // group 0 uses tiles 0..3, group 1 tiles 1..3
                bf16x8_t h[kBMaxW], l[kBMaxW];
#pragma unroll
                for (int a = 0; a < kBMaxW; ++a) {
                    if (a < Wi && (pg == 0 || a >= 1)) {
                        h[a] = operand(hiA, a, ks);
                        if (SPLIT) l[a] = operand(loA, a, ks);
                    }
                }
                if (pg == 0) {
#pragma unroll
                    for (int t = 0; t < 5; ++t)
                        if (dg_b(0, t) < Wi)
                            acc[t] = mfma3<SPLIT>(acc[t], h[dg_a(0, t)], l[dg_a(0, t)], h[dg_b(0, t)], l[dg_b(0, t)]);
                } else {
#pragma unroll
                    for (int t = 0; t < 5; ++t)
                        if (dg_b(1, t) < Wi)
                            acc[t] = mfma3<SPLIT>(acc[t], h[dg_a(1, t)], l[dg_a(1, t)], h[dg_b(1, t)], l[dg_b(1, t)]);
                }
            } else {
                bf16x8_t ah[2], al[2], bh[kBMaxW], bl[kBMaxW];
#pragma unroll
                for (int a = 0; a < 2; ++a) {
                    if (2 * pg + a < Wi) {
                        ah[a] = operand(hiA, 2 * pg + a, ks);
                        if (SPLIT) al[a] = operand(loA, 2 * pg + a, ks);
                    }
                }
#pragma unroll
                for (int b = 0; b < kBMaxW; ++b) {
                    if (b < Wj) {
                        bh[b] = operand(hiB, b, ks);
                        if (SPLIT) bl[b] = operand(loB, b, ks);
                    }
                }
#pragma unroll
                for (int a = 0; a < 2; ++a)
#pragma unroll
                    for (int b = 0; b < kBMaxW; ++b)
                        if (2 * pg + a < Wi && b < Wj)
                            acc[4 * a + b] = mfma3<SPLIT>(acc[4 * a + b], ah[a], al[a], bh[b], bl[b]);
            }
        }
    };

    if (nchunks > 0) load_chunk(0);
    for (int c = 0; c < nchunks; ++c) {
        stage_chunk();
        __syncthreads();
        if (c + 1 < nchunks) load_chunk(c + 1);   // in flight during the MFMAs
        mma_chunk();
        __syncthreads();
    }

    // Sum the waves' accumulators of each tile pair in wave order and write
    // the FP32 partial.  v_mfma_f32_32x32x16_bf16 leaves
    // D[8 (r / 4) + 4 (lane / 32) + r % 4][lane % 32] in element r.
    float *red = reinterpret_cast<float *>(smem_raw);   // kBWaves x 1024 floats
    const size_t part_id = (size_t)k * g.nsplit + s;
    auto put = [&](const f32x16_t &v, int slot) {
#pragma unroll
        for (int r = 0; r < 16; ++r)
            red[slot * 1024 + (8 * (r / 4) + 4 * (lane / 32) + (r % 4)) * kBTile + (lane % 32)] = v[r];
    };
    auto emit = [&](int ti, int tj, int nw) {
        __syncthreads();
        float *dst = partial + (part_id * g.ntp + tile_pair_index(ti, tj, g.T)) * (kBTile * kBTile);
        for (int e = threadIdx.x; e < 1024; e += kBThreads) {
            float v = red[e];
            for (int w = 1; w < nw; ++w) v += red[w * 1024 + e];
            dst[e] = v;
        }
        __syncthreads();
    };
#pragma unroll
    for (int grp = 0; grp < 2; ++grp) {
#pragma unroll
        for (int t = 0; t < NSLOT; ++t) {
            const int a = DIAG ? dg_a(grp, t) : 2 * grp + t / 4;
            const int b = DIAG ? dg_b(grp, t) : t % 4;
            if (DIAG ? (b < Wi) : (a < Wi && b < Wj)) {
                if (pg == grp) put(acc[t], wave % 2);
                emit(I * g.W + a, J * g.W + b, 2);
            }
        }
    }

    // FP64 diagonal, X^T y, y^T y: the 8 row groups of a column are combined
    // in order; pvec = [split][diag p | xy p], pscal = [split][yy, n]
    if (diag) {
        double *vred = reinterpret_cast<double *>(smem_raw);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            vred[rg * kBPanel + lc + 32 * j] = sd[j];
            vred[8 * kBPanel + rg * kBPanel + lc + 32 * j] = sxy[j];
        }
        if (lc == 0) vred[16 * kBPanel + rg] = syy;
        __syncthreads();
        if (threadIdx.x < kBPanel) {
            const int col = I * g.W * kBTile + threadIdx.x;
            double d = 0.0, b = 0.0;
            for (int r = 0; r < 8; ++r) {
                d += vred[r * kBPanel + threadIdx.x];
                b += vred[8 * kBPanel + r * kBPanel + threadIdx.x];
            }
            if (col < g.p) {
                pvec[part_id * 2 * g.p + col] = d;
                pvec[part_id * 2 * g.p + g.p + col] = b;
            }
        }
        if (first_block && threadIdx.x == 0) {
            double t = 0.0;
            for (int r = 0; r < 8; ++r) t += vred[16 * kBPanel + r];
            pscal[part_id * 2] = t;
            pscal[part_id * 2 + 1] = (double)count;
        }
    }
}

// One launch for the whole cross-split reduction: thread e of fold k sums
// the splits of entry e (tiles, then diagonal and X^T y, then y^T y and n)
// in split order and adds the result into the running statistics; upper
// tile entries are mirrored so G stays exactly symmetric.
__global__ void gram_bf16_reduce_kernel(GramGeom g, const float *__restrict__ partial,
                                        const double *__restrict__ pvec,
                                        const double *__restrict__ pscal, double *__restrict__ Gk,
                                        double *__restrict__ bk, double *__restrict__ yyk,
                                        int64_t *__restrict__ nk)
{
    const int p = g.p, S = g.nsplit;
    const size_t tile = kBTile * kBTile;
    const size_t Et = (size_t)g.ntp * tile;
    const size_t per_k = Et + 2 * (size_t)p + 1;
    const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (size_t)g.K * per_k) return;
    const int k = (int)(idx / per_k);
    const size_t e = idx % per_k;
    if (e < Et) {
        const int te = (int)(e % tile);
        const int tp = (int)(e / tile);
        int ti, tj;
        tile_pair_decode(tp, g.T, ti, tj);
        const int ei = te / kBTile, ej = te % kBTile;
        if (ti == tj && ei >= ej) return;         // diagonal from FP64; lower half mirrored
        const int i = ti * kBTile + ei, j = tj * kBTile + ej;
        if (i >= p || j >= p) return;
        const float *src = partial + (size_t)k * S * Et + e;
        double sum = 0.0;
        for (int sp = 0; sp < S; ++sp) sum += (double)src[(size_t)sp * Et];
        double *G = Gk + (size_t)k * p * p;
        G[(size_t)i * p + j] += sum;
        G[(size_t)j * p + i] += sum;
    } else if (e < Et + 2 * (size_t)p) {
        const size_t v = e - Et;
        const double *src = pvec + (size_t)k * S * 2 * p + v;
        double sum = 0.0;
        for (int sp = 0; sp < S; ++sp) sum += src[(size_t)sp * 2 * p];
        if (v < (size_t)p) Gk[(size_t)k * p * p + v * p + v] += sum;
        else bk[(size_t)k * p + (v - p)] += sum;
    } else {
        const double *src = pscal + (size_t)k * S * 2;
        double yy = 0.0, cnt = 0.0;
        for (int sp = 0; sp < S; ++sp) {
            yy += src[(size_t)sp * 2];
            cnt += src[(size_t)sp * 2 + 1];
        }
        yyk[k] += yy;
        nk[k] += (int64_t)cnt;
    }
}

static GramGeom plan_bf16(int p, int K, int64_t n)
{
    GramGeom g{};
    g.p = p;
    g.pa = p;
    g.tile = kBTile;
    g.T = (p + kBTile - 1) / kBTile;
    g.W = std::min(g.T, kBMaxW);
    g.nsb = (g.T + g.W - 1) / g.W;
    g.npsb = g.nsb * (g.nsb + 1) / 2;
    g.ntp = g.T * (g.T + 1) / 2;
    g.K = K;
    g.rk = kBRows;
    // about two workgroups per CU; with folds, splits are whole 4096-row blocks
    const int64_t target = 512;
    int64_t ns = std::max<int64_t>(1, (target + (int64_t)K * g.npsb - 1) / ((int64_t)K * g.npsb));
    int64_t rps = (n + ns - 1) / ns;
    const int64_t quantum = (K == 1) ? kBRows : 4096;
    rps = std::max<int64_t>(quantum, (rps + quantum - 1) / quantum * quantum);
    g.rows_per_split = rps;
    g.nsplit = (int)std::max<int64_t>(1, (n + rps - 1) / rps);
    return g;
}

static size_t bf16_lds_bytes(const GramGeom &g, bool diag)
{
    (void)g;
    const int npanels = diag ? 2 : 4;
    const size_t panels = (size_t)npanels * kBPanel * kBPitch * sizeof(__bf16);
    const size_t red = std::max((size_t)kBWaves * 1024 * sizeof(float),
                                (size_t)(16 * kBPanel + 8) * sizeof(double));
    return std::max(panels, red);
}

int launch_gram_bf16(oem_gram_s *h, const void *Xv, int64_t n, int64_t ldx, const double *y,
                     int64_t row_offset, const uint8_t *foldid, hipStream_t s)
{
    if (h->xdt != OEM_X_F32) return fail(OEM_E_INVAL, "the BF16 Gram forms take FP32 X");
    const float *X = static_cast<const float *>(Xv);
    const GramGeom g = plan_bf16(h->p, h->K, n);
    RowSource rs;
    int rc = build_row_lists(h, g, n, row_offset, foldid, rs, s);
    if (rc) return rc;
    const size_t S = g.nsplit, K = g.K;
    const size_t Et = (size_t)g.ntp * kBTile * kBTile;
    const size_t parts = K * S;
    const size_t bytes = parts * Et * sizeof(float) + parts * (2 * g.p + 2) * sizeof(double) + 64;
    rc = h->partial.ensure(bytes);
    if (rc) return rc;
    float *part = h->partial.as<float>();
    double *pvec = reinterpret_cast<double *>(part + parts * Et);
    double *pscal = pvec + parts * 2 * g.p;
    const bool split = (h->prec == OEM_SPLIT_BF16);
    {
        const size_t lds = bf16_lds_bytes(g, true);
        auto kern = split ? gram_bf16_kernel<true, true> : gram_bf16_kernel<false, true>;
        OEM_HIP_CHECK(hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
        hipLaunchKernelGGL(kern, dim3(g.K * g.nsplit * g.nsb), dim3(kBThreads), lds, s, X, n, ldx, y, g, rs,
                           part, pvec, pscal);
        OEM_HIP_CHECK(hipGetLastError());
    }
    if (g.npsb > g.nsb) {
        const size_t lds = bf16_lds_bytes(g, false);
        auto kern = split ? gram_bf16_kernel<true, false> : gram_bf16_kernel<false, false>;
        OEM_HIP_CHECK(hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
        hipLaunchKernelGGL(kern, dim3(g.K * g.nsplit * (g.npsb - g.nsb)), dim3(kBThreads), lds, s, X, n, ldx, y,
                           g, rs, part, pvec, pscal);
        OEM_HIP_CHECK(hipGetLastError());
    }
    const size_t total = K * (Et + 2 * (size_t)g.p + 1);
    hipLaunchKernelGGL(gram_bf16_reduce_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, g,
                       part, pvec, pscal, h->Gk.as<double>(), h->bk.as<double>(), h->yyk.as<double>(),
                       h->nk.as<int64_t>());
    OEM_HIP_CHECK(hipGetLastError());
    return OEM_OK;
}

} // namespace oem
