// Streaming Gram pass (Section 3: per-fold X_k^T X_k and X_k^T y_k in one
// pass over the rows) for gfx950.
//
// FP64 form: the augmented matrix [X y] is staged through LDS in 64-row
// chunks and multiplied on the FP64 matrix cores (v_mfma_f64_16x16x4f64); FP32
// X is kept FP32 in LDS and widened (exactly) when an operand is read, y is
// kept FP64.  The upper triangle of [X y]^T [X y] holds X^T X, X^T y
// (column p) and y^T y (corner), so one contraction gives every statistic.
//
// Work decomposition: the upper triangle of 16x16 tiles is cut into
// super-blocks of W x W tiles; a workgroup owns one (fold, row split,
// super-block pair) and streams that split's rows of its fold (a
// precomputed ordered row list), so every row is fetched once per
// super-block pair.  Each thread loads an 8-row x 4-column block per chunk,
// and the next chunk's loads are issued before the current chunk's MFMAs.
// Workgroups sharing a row split are numbered so that round-robin dispatch
// places them on one XCD, where they share that XCD's L2.  Partial tiles are
// summed over splits in a fixed order (deterministic, no floating-point
// atomics).
#include "gram_common.h"

namespace oem {

typedef double d4_t __attribute__((ext_vector_type(4)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));

constexpr int kGramThreads = 256;
constexpr int kGramWaves = kGramThreads / kWave;
constexpr int kMaxW = 8;                                   // tiles per super-block side
constexpr int kPanelCols = 16 * kMaxW;                     // 128
constexpr int kRows = 64;                                  // rows per chunk (16 MFMA k-steps)
constexpr int kMaxSlots = (kMaxW * kMaxW + kGramWaves - 1) / kGramWaves;  // tile pairs per wave

// LDS row pitch (elements) of a staged panel: 128 + 4 keeps 16-byte rows
// aligned and shifts successive rows across banks.
constexpr int kPitch = kPanelCols + 4;

// Thread (c4, rg) loads rows 8 rg .. 8 rg + 7, columns 4 c4 .. 4 c4 + 3 of a
// panel and stores them row-major into LDS (elements of the input type).
template <typename XT, bool VEC>
__device__ inline void load_rows(XT (&b)[8][4], const XT *__restrict__ X, int64_t ldx, int p, int col,
                                 const int64_t *rows, const bool *ok)
{
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        if constexpr (VEC) {
            if (ok[e] && col + 3 < p) {
                const f32x4_t v = *reinterpret_cast<const f32x4_t *>(X + rows[e] * ldx + col);
                b[e][0] = v[0];
                b[e][1] = v[1];
                b[e][2] = v[2];
                b[e][3] = v[3];
                continue;
            }
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) b[e][j] = (ok[e] && col + j < p) ? X[rows[e] * ldx + col + j] : XT(0);
    }
}

template <typename XT>
__device__ inline void store_rows(const XT (&b)[8][4], XT *panel, int c4, int rg)
{
#pragma unroll
    for (int e = 0; e < 8; ++e)
#pragma unroll
        for (int j = 0; j < 4; ++j) panel[(8 * rg + e) * kPitch + 4 * c4 + j] = b[e][j];
}

template <typename XT, bool VEC>
__global__ __launch_bounds__(kGramThreads) void gram_f64_kernel(
    const XT *__restrict__ X, int64_t n, int64_t ldx, const double *__restrict__ y, GramGeom g,
    RowSource rs, double *__restrict__ partial, double *__restrict__ pscal)
{
    extern __shared__ double smem[];
    const int lane = threadIdx.x % kWave;
    const int wave = threadIdx.x / kWave;
    const int c4 = threadIdx.x % 32, rg = threadIdx.x / 32;

    const int L = xcd_logical(blockIdx.x, gridDim.x);
    const int q = L % g.npsb;
    const int rest = L / g.npsb;
    const int s = rest % g.nsplit;
    const int k = rest / g.nsplit;
    int I = 0, J = 0;
    sb_pair_decode(q, g.nsb, I, J);
    const int Wi = min(g.W, g.T - I * g.W);
    const int Wj = min(g.W, g.T - J * g.W);
    const bool diag = (I == J);

    double *ylds = smem;                                   // kRows
    XT *A = reinterpret_cast<XT *>(smem + kRows);          // kRows x kPitch
    XT *B = diag ? A : A + kRows * kPitch;

    const int npairs = diag ? Wi * (Wi + 1) / 2 : Wi * Wj;
    int ta[kMaxSlots], tb[kMaxSlots];
#pragma unroll
    for (int t = 0; t < kMaxSlots; ++t) {
        const int m = wave + kGramWaves * t;
        int a = 0, b = 0;
        if (m < npairs) {
            if (diag) {
                int mm = m;
                for (a = 0; a < Wi; ++a) {
                    const int cnt = Wi - a;
                    if (mm < cnt) { b = a + mm; break; }
                    mm -= cnt;
                }
            } else {
                a = m / Wj;
                b = m % Wj;
            }
        }
        ta[t] = a;
        tb[t] = b;
    }
    const int nslots = (npairs > wave) ? (npairs - wave + kGramWaves - 1) / kGramWaves : 0;

    d4_t acc[kMaxSlots];
#pragma unroll
    for (int t = 0; t < kMaxSlots; ++t) acc[t] = d4_t{0.0, 0.0, 0.0, 0.0};

    int64_t first, count;
    const int32_t *list;
    rows_of(g, rs, n, k, s, first, count, list);
    const int nchunks = (int)((count + kRows - 1) / kRows);
    const int baseA = I * g.W * 16, baseB = J * g.W * 16;

    XT ba[8][4], bb[8][4];
    double yv = 0.0;
    auto load_chunk = [&](int c) {
        int64_t rows[8];
        bool ok[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int64_t i = (int64_t)c * kRows + 8 * rg + e;
            ok[e] = i < count;
            rows[e] = ok[e] ? row_at(first, list, i) : 0;
        }
        load_rows<XT, VEC>(ba, X, ldx, g.p, baseA + 4 * c4, rows, ok);
        if (!diag) load_rows<XT, VEC>(bb, X, ldx, g.p, baseB + 4 * c4, rows, ok);
        if (threadIdx.x < kRows) {
            const int64_t i = (int64_t)c * kRows + threadIdx.x;
            yv = (i < count) ? y[row_at(first, list, i)] : 0.0;
        }
    };
    // operand of augmented column `col` (global index) at chunk row r
    auto aug = [&](const XT *panel, int base, int r, int cl) -> double {
        const int col = base + cl;
        if (col < g.p) return (double)panel[r * kPitch + cl];
        return (col == g.p) ? ylds[r] : 0.0;
    };
    auto mma_chunk = [&]() {
        for (int kk = 0; kk < kRows / 4; ++kk) {
            const int r = 4 * kk + lane / 16;
#pragma unroll
            for (int t = 0; t < kMaxSlots; ++t) {
                if (t < nslots) {
                    const double a = aug(A, baseA, r, ta[t] * 16 + (lane % 16));
                    const double b = aug(B, baseB, r, tb[t] * 16 + (lane % 16));
                    acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[t], 0, 0, 0);
                }
            }
        }
    };

    if (nchunks > 0) load_chunk(0);
    for (int c = 0; c < nchunks; ++c) {
        store_rows(ba, A, c4, rg);
        if (!diag) store_rows(bb, B, c4, rg);
        if (threadIdx.x < kRows) ylds[threadIdx.x] = yv;
        __syncthreads();
        if (c + 1 < nchunks) load_chunk(c + 1);   // in flight during the MFMAs
        mma_chunk();
        __syncthreads();
    }

    // v_mfma_f64_16x16x4f64 leaves D[4 r + lane / 16][lane % 16] in element r.
    const size_t part_id = (size_t)k * g.nsplit + s;
#pragma unroll
    for (int t = 0; t < kMaxSlots; ++t) {
        if (t < nslots) {
            const int ti = I * g.W + ta[t], tj = J * g.W + tb[t];
            double *dst = partial + (part_id * g.ntp + tile_pair_index(ti, tj, g.T)) * 256;
#pragma unroll
            for (int r = 0; r < 4; ++r) dst[(4 * r + lane / 16) * 16 + (lane % 16)] = acc[t][r];
        }
    }
    if (q == 0 && threadIdx.x == 0) pscal[part_id] = (double)count;
}

// Add the reduced tiles of [X y]^T [X y] into G, X^T y and y^T y; the upper
// triangle is mirrored so G stays exactly symmetric.
__global__ void gram_f64_scatter_kernel(GramGeom g, const double *__restrict__ tiles,
                                        const double *__restrict__ cnt, double *__restrict__ Gk,
                                        double *__restrict__ bk, double *__restrict__ yyk,
                                        int64_t *__restrict__ nk)
{
    const size_t per_k = (size_t)g.ntp * 256;
    const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx < (size_t)g.K) nk[idx] += (int64_t)cnt[idx];
    if (idx >= (size_t)g.K * per_k) return;
    const int e = (int)(idx % 256);
    const int tp = (int)((idx / 256) % g.ntp);
    const int k = (int)(idx / per_k);
    int ti, tj;
    tile_pair_decode(tp, g.T, ti, tj);
    const int ei = e / 16, ej = e % 16;
    if (ti == tj && ei > ej) return;
    const int i = ti * 16 + ei, j = tj * 16 + ej;
    if (i > g.p || j > g.p) return;
    const double sum = tiles[idx];
    const int p = g.p;
    if (j < p) {
        double *G = Gk + (size_t)k * p * p;
        G[(size_t)i * p + j] += sum;
        if (i != j) G[(size_t)j * p + i] += sum;
    } else if (i < p) {
        bk[(size_t)k * p + i] += sum;
    } else {
        yyk[k] += sum;
    }
}

__global__ void fill_f64_kernel(double *p, size_t n, double v)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void fill_i64_kernel(int64_t *p, size_t n, int64_t v)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void scale_f64_kernel(double *p, size_t n, double v)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        p[i] *= v;
}

int launch_scale_f64(double *p, size_t n, double v, hipStream_t s)
{
    if (n == 0) return OEM_OK;
    int blocks = (int)std::min<size_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(scale_f64_kernel, dim3(blocks), dim3(256), 0, s, p, n, v);
    OEM_HIP_CHECK(hipGetLastError());
    return OEM_OK;
}

int launch_fill_f64(double *p, size_t n, double v, hipStream_t s)
{
    if (n == 0) return OEM_OK;
    int blocks = (int)std::min<size_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(fill_f64_kernel, dim3(blocks), dim3(256), 0, s, p, n, v);
    OEM_HIP_CHECK(hipGetLastError());
    return OEM_OK;
}

int launch_fill_i64(int64_t *p, size_t n, int64_t v, hipStream_t s)
{
    if (n == 0) return OEM_OK;
    int blocks = (int)std::min<size_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(fill_i64_kernel, dim3(blocks), dim3(256), 0, s, p, n, v);
    OEM_HIP_CHECK(hipGetLastError());
    return OEM_OK;
}

static GramGeom plan_f64(int prec, int p, int K, int64_t n)
{
    GramGeom g{};
    g.p = p;
    g.pa = p + 1;
    g.tile = 16;
    g.T = (g.pa + 15) / 16;
    g.W = std::min(g.T, kMaxW);
    g.nsb = (g.T + g.W - 1) / g.W;
    g.npsb = g.nsb * (g.nsb + 1) / 2;
    g.ntp = g.T * (g.T + 1) / 2;
    g.K = K;
    g.rk = kRows;
    const int64_t target = gram_target(prec, K, p, n);
    int64_t ns = std::max<int64_t>(1, (target + (int64_t)K * g.npsb - 1) / ((int64_t)K * g.npsb));
    int64_t rps = (n + ns - 1) / ns;
    const int64_t quantum = (K == 1) ? kRows : 4096;
    rps = std::max<int64_t>(quantum, (rps + quantum - 1) / quantum * quantum);
    g.rows_per_split = rps;
    g.nsplit = (int)std::max<int64_t>(1, (n + rps - 1) / rps);
    return g;
}

template <typename XT, bool VEC>
static int launch_f64_t(const GramGeom &g, const XT *X, int64_t n, int64_t ldx, const double *y,
                        const RowSource &rs, double *part, double *pscal, hipStream_t s)
{
    const int npanels = (g.nsb == 1) ? 1 : 2;
    const size_t lds = kRows * sizeof(double) + (size_t)npanels * kRows * kPitch * sizeof(XT);
    const int blocks = g.K * g.nsplit * g.npsb;
    auto kern = gram_f64_kernel<XT, VEC>;
    OEM_HIP_CHECK(hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    hipLaunchKernelGGL(kern, dim3(blocks), dim3(kGramThreads), lds, s, X, n, ldx, y, g, rs, part, pscal);
    OEM_HIP_CHECK(hipGetLastError());
    return OEM_OK;
}

int launch_gram(oem_gram_s *h, const void *X, int64_t n, int64_t ldx, const double *y,
                int64_t row_offset, const uint8_t *foldid, hipStream_t s)
{
    if (h->prec != OEM_FP64) return launch_gram_bf16(h, X, n, ldx, y, row_offset, foldid, s);
    const GramGeom g = plan_f64(h->prec, h->p, h->K, n);
    RowSource rs;
    int rc = build_row_lists(h, g, n, row_offset, foldid, rs, s);
    if (rc) return rc;
    const size_t K = g.K, S = g.nsplit;
    const size_t E = (size_t)g.ntp * 256;
    rc = h->partial.ensure((K * S * E + K * S + 8) * sizeof(double));
    if (rc) return rc;
    double *part = h->partial.as<double>();
    double *pscal = part + K * S * E;
    const size_t red = reduce_tmp_doubles(g.K, g.nsplit, E) + K * (E + 1) + 8;
    rc = h->redtmp.ensure(red * sizeof(double));
    if (rc) return rc;
    if (h->xdt == OEM_X_F32) {
        const float *Xf = static_cast<const float *>(X);
        const bool vec = ((reinterpret_cast<uintptr_t>(Xf) & 15) == 0) && (ldx % 4 == 0);
        rc = vec ? launch_f64_t<float, true>(g, Xf, n, ldx, y, rs, part, pscal, s)
                 : launch_f64_t<float, false>(g, Xf, n, ldx, y, rs, part, pscal, s);
    } else {
        rc = launch_f64_t<double, false>(g, static_cast<const double *>(X), n, ldx, y, rs, part, pscal, s);
    }
    if (rc) return rc;
    double *tmp = h->redtmp.as<double>();
    double *out_tiles = tmp + reduce_tmp_doubles(g.K, g.nsplit, E);
    double *out_cnt = out_tiles + K * E;
    rc = reduce_splits_f64(part, g.K, g.nsplit, E, tmp, out_tiles, s);
    rc = rc ? rc : reduce_splits_f64(pscal, g.K, g.nsplit, 1, tmp, out_cnt, s);
    if (rc) return rc;
    const size_t total = K * E;
    hipLaunchKernelGGL(gram_f64_scatter_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, g,
                       out_tiles, out_cnt, h->Gk.as<double>(), h->bk.as<double>(), h->yyk.as<double>(),
                       h->nk.as<int64_t>());
    OEM_HIP_CHECK(hipGetLastError());
    return OEM_OK;
}

} // namespace oem
