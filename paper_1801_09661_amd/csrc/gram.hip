// Streaming Gram pass (Section 3: per-fold X_k^T X_k and X_k^T y_k in one
// pass over the rows) for gfx950.
//
// FP64 form: X is staged through LDS in 64-row chunks (FP32 X stays FP32 in
// LDS and is widened, exactly, when an operand is read) and X^T X is formed on
// the FP64 matrix cores (v_mfma_f64_16x16x4f64).  X^T y and y^T y are
// accumulated in FP64 on the vector units from the loaded values, by the
// workgroups of the diagonal super-blocks.
//
// Work decomposition: the upper triangle of 16x16 tiles is cut into
// super-blocks of W x W tiles; a workgroup owns one (fold, row split,
// super-block pair) and streams that split's rows (contiguous rows with one
// fold, an ordered row list per (fold, split) with several), so every row is
// fetched once per super-block pair.  Thread (q, rg) loads columns
// 4q .. 4q + 3 of 8 rows (16-byte loads whatever the row pitch) and the next
// chunk's loads are issued before the current chunk's MFMAs; rows past the
// end of the split are read as copies of its last row and cleared before
// staging.  Workgroups sharing a row split are numbered so that round-robin
// dispatch places them on one XCD, where they share that XCD's L2.  Partial
// tiles are summed over splits in a fixed order (deterministic, no
// floating-point atomics).
#include "gram_common.h"

namespace oem {

typedef double d4_t __attribute__((ext_vector_type(4)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));
typedef double f64x2_t __attribute__((ext_vector_type(2)));

constexpr int kGramThreads = 256;
constexpr int kGramWaves = kGramThreads / kWave;
constexpr int kMaxW = 8;                                   // tiles per super-block side
constexpr int kPanelCols = 16 * kMaxW;                     // 128
constexpr int kRows = 64;                                  // rows per chunk (16 MFMA k-steps)
constexpr int kMaxSlots = (kMaxW * kMaxW + kGramWaves - 1) / kGramWaves;  // tile pairs per wave

// LDS row pitch (elements) of a staged row-major panel: 16-byte aligned rows,
// successive rows shifted across banks.
template <typename XT> constexpr int panel_pitch() { return sizeof(XT) == 4 ? kPanelCols + 4 : kPanelCols + 2; }

// Thread (q, rg): columns col .. col + 3 of the 8 rows `row`.  Columns at or
// past p read a valid column instead (they only feed discarded tile entries).
template <typename XT, bool VEC>
__device__ inline void load_block64(XT (&x)[8][4], const XT *__restrict__ X, int64_t ldx, int p, int col,
                                    const int64_t (&row)[8])
{
    // 16-byte loads need only element alignment on gfx950 (column choice:
    // gram_col_plan).
    const GramColPlan cp = gram_col_plan(VEC, col, p);
    if (cp.vec) {
        const int cv = cp.first;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const XT *src = X + row[e] * ldx + cv;
            if constexpr (sizeof(XT) == 4) {
                const f32x4_t v = *reinterpret_cast<const f32x4_t *>(src);
#pragma unroll
                for (int j = 0; j < 4; ++j) x[e][j] = v[j];
            } else {
                const f64x2_t v0 = *reinterpret_cast<const f64x2_t *>(src);
                const f64x2_t v1 = *reinterpret_cast<const f64x2_t *>(src + 2);
                x[e][0] = v0[0];
                x[e][1] = v0[1];
                x[e][2] = v1[0];
                x[e][3] = v1[1];
            }
        }
    } else {
        int cj[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) cj[j] = gram_col_read(cp, col, j, p);
#pragma unroll
        for (int e = 0; e < 8; ++e)
#pragma unroll
            for (int j = 0; j < 4; ++j) x[e][j] = X[row[e] * ldx + cj[j]];
    }
}

// Rows of a sparse X in compressed sparse row form (Section 5.8): row r
// stores entries t in [rowptr[r], rowptr[r + 1]) at columns col[t] with
// values val[t].  Entry ranges are clamped to [0, nnz), so a malformed
// rowptr cannot make a load leave the arrays.
template <typename XT> struct CsrRows {
    const int64_t *rowptr;
    const int32_t *col;
    const XT *val;
    int64_t nnz;
};

// The same thread block as load_block64 from CSR rows: columns col .. col + 3
// of the 8 rows, zero where a row stores no entry (repeated entries add).
// Registers end up as in the dense loader for every column below p, so the
// MFMA sums equal those of the densified rows bit for bit.
template <typename XT>
__device__ inline void load_block64_csr(XT (&x)[8][4], const CsrRows<XT> &A, int col, const int64_t (&row)[8])
{
#pragma unroll
    for (int e = 0; e < 8; ++e)
#pragma unroll
        for (int j = 0; j < 4; ++j) x[e][j] = XT(0);
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        int64_t t0 = A.rowptr[row[e]], t1 = A.rowptr[row[e] + 1];
        t0 = t0 < 0 ? 0 : (t0 > A.nnz ? A.nnz : t0);
        t1 = t1 < t0 ? t0 : (t1 > A.nnz ? A.nnz : t1);
        for (int64_t t = t0; t < t1; ++t) {
            const int c = A.col[t] - col;
            const XT v = A.val[t];
#pragma unroll
            for (int j = 0; j < 4; ++j)
                if (c == j) x[e][j] += v;
        }
    }
}

template <typename XT>
__device__ inline void store_block64(const XT (&x)[8][4], XT *panel, int q, int rg)
{
    constexpr int PP = panel_pitch<XT>();
#pragma unroll
    for (int e = 0; e < 8; ++e)
#pragma unroll
        for (int j = 0; j < 4; ++j) panel[(8 * rg + e) * PP + 4 * q + j] = x[e][j];
}

// WGT: row weights w (n): the tiles accumulate sum_i w_i x_i x_i^T (the
// weighted Gram of a Newton step, Section 4); the other sums stay unweighted.
template <typename XT, bool LIST, bool VEC, bool CSR, bool WGT>
__global__ __launch_bounds__(kGramThreads) void gram_f64_kernel(
    const XT *__restrict__ X, int64_t n, int64_t ldx, const double *__restrict__ y, GramGeom g,
    RowSource rs, double *__restrict__ partial, double *__restrict__ pvec, double *__restrict__ pscal,
    CsrRows<XT> csr, const double *__restrict__ wts)
{
    constexpr int PP = panel_pitch<XT>();
    extern __shared__ double smem[];
    const int lane = threadIdx.x % kWave;
    const int wave = threadIdx.x / kWave;
    const int q4 = threadIdx.x % 32, rg = threadIdx.x / 32;

    const int L = xcd_logical(blockIdx.x, gridDim.x);
    const int qq = L % g.npsb;
    const int rest = L / g.npsb;
    const int s = rest % g.nsplit;
    const int k = rest / g.nsplit;
    int I = 0, J = 0;
    sb_pair_decode(qq, g.nsb, I, J);
    const int Wi = min(g.W, g.T - I * g.W);
    const int Wj = min(g.W, g.T - J * g.W);
    const bool diag = (I == J);
    const bool first_block = (qq == 0);

    XT *A = reinterpret_cast<XT *>(smem);
    XT *B = diag ? A : A + kRows * PP;
    // row weights of the staged chunk (WGT), after the panels
    double *wl = reinterpret_cast<double *>(A + (g.nsb == 1 ? 1 : 2) * kRows * PP);

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
    const int colA = I * g.W * 16 + 4 * q4, colB = J * g.W * 16 + 4 * q4;
    double sxy[4] = {0.0, 0.0, 0.0, 0.0}, syy = 0.0;
    double sx[4] = {0.0, 0.0, 0.0, 0.0}, sy = 0.0;   // column sums and sum of y

    XT xa[8][4], xb[8][4];
    double yv[8];
    double wv[8];
    int32_t nidx[8];
    auto load_index = [&](int c) {
        if constexpr (LIST) {
#pragma unroll
            for (int e = 0; e < 8; ++e) nidx[e] = list[min((int64_t)c * kRows + 8 * rg + e, count - 1)];
        }
    };
    auto load_chunk = [&](int c) {
        int64_t row[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            if constexpr (LIST) row[e] = nidx[e];
            else row[e] = first + min((int64_t)c * kRows + 8 * rg + e, count - 1);
        }
        if constexpr (CSR) {
            load_block64_csr<XT>(xa, csr, colA, row);
            if (!diag) load_block64_csr<XT>(xb, csr, colB, row);
        } else {
            load_block64<XT, VEC>(xa, X, ldx, g.p, colA, row);
            if (!diag) load_block64<XT, VEC>(xb, X, ldx, g.p, colB, row);
        }
        if (diag) {
#pragma unroll
            for (int e = 0; e < 8; ++e) yv[e] = y[row[e]];
        }
        if constexpr (WGT) {
#pragma unroll
            for (int e = 0; e < 8; ++e) wv[e] = wts[row[e]];
        }
    };
    auto clear_tail = [&](int c) {
        const int64_t r0 = (int64_t)c * kRows + 8 * rg;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            if (r0 + e >= count) {
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    xa[e][j] = XT(0);
                    xb[e][j] = XT(0);
                }
                yv[e] = 0.0;
            }
        }
    };
    auto stage_chunk = [&]() {
        store_block64<XT>(xa, A, q4, rg);
        if (!diag) store_block64<XT>(xb, B, q4, rg);
        if constexpr (WGT) {
            if (q4 == 0) {
#pragma unroll
                for (int e = 0; e < 8; ++e) wl[8 * rg + e] = wv[e];
            }
        }
        if (diag) {
#pragma unroll
            for (int e = 0; e < 8; ++e) {
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    sxy[j] += (double)xa[e][j] * yv[e];
                    sx[j] += (double)xa[e][j];
                }
                syy += yv[e] * yv[e];
                sy += yv[e];
            }
        }
    };
    auto mma_chunk = [&]() {
#pragma unroll 4
        for (int kk = 0; kk < kRows / 4; ++kk) {
            const int r = 4 * kk + lane / 16;
#pragma unroll
            for (int t = 0; t < kMaxSlots; ++t) {
                if (t < nslots) {
                    double a = (double)A[r * PP + ta[t] * 16 + (lane % 16)];
                    if constexpr (WGT) a *= wl[r];
                    const double b = (double)B[r * PP + tb[t] * 16 + (lane % 16)];
                    acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[t], 0, 0, 0);
                }
            }
        }
    };

    if (nchunks > 0) {
        load_index(0);
        load_chunk(0);
        load_index(1);
    }
    for (int c = 0; c < nchunks; ++c) {
        if ((int64_t)(c + 1) * kRows > count) clear_tail(c);
        stage_chunk();
        __syncthreads();
        if (c + 1 < nchunks) {
            load_chunk(c + 1);   // in flight during the MFMAs
            load_index(c + 2);
        }
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
    // X^T y, column sums, y^T y and sum y: the 8 row groups of a column
    // combined in order; pvec = [part][xy p | colsum p], pscal = [part][yy, n, sum y]
    if (diag) {
        double *vred = smem;   // 16 x kPanelCols + 16
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            vred[rg * kPanelCols + 4 * q4 + j] = sxy[j];
            vred[8 * kPanelCols + rg * kPanelCols + 4 * q4 + j] = sx[j];
        }
        if (q4 == 0) {
            vred[16 * kPanelCols + rg] = syy;
            vred[16 * kPanelCols + 8 + rg] = sy;
        }
        __syncthreads();
        if (threadIdx.x < kPanelCols) {
            const int col = I * g.W * 16 + threadIdx.x;
            double b = 0.0, c = 0.0;
            for (int r = 0; r < 8; ++r) {
                b += vred[r * kPanelCols + threadIdx.x];
                c += vred[8 * kPanelCols + r * kPanelCols + threadIdx.x];
            }
            if (col < g.p) {
                pvec[part_id * 2 * g.p + col] = b;
                pvec[part_id * 2 * g.p + g.p + col] = c;
            }
        }
        if (first_block && threadIdx.x == 0) {
            double t = 0.0, u = 0.0;
            for (int r = 0; r < 8; ++r) {
                t += vred[16 * kPanelCols + r];
                u += vred[16 * kPanelCols + 8 + r];
            }
            pscal[part_id * 3] = t;
            pscal[part_id * 3 + 1] = (double)count;
            pscal[part_id * 3 + 2] = u;
        }
    }
}

// Finish the pass: sum each statistic over the row splits (fixed order) and
// add it into the running sums: upper-triangle tile entries mirrored into the
// lower triangle (G stays exactly symmetric), then X^T y and the column sums,
// then y^T y, n and sum y.  Grid (statistic blocks of 64, folds).
__global__ __launch_bounds__(kFinishThreads) void gram_f64_finish_kernel(
    GramGeom g, const double *__restrict__ tiles, const double *__restrict__ vec,
    const double *__restrict__ scal, double *__restrict__ Gk, double *__restrict__ bk,
    double *__restrict__ yyk, int64_t *__restrict__ nk, double *__restrict__ csk,
    double *__restrict__ ysk)
{
    __shared__ double red[kFinishThreads];
    const int p = g.p, S = g.nsplit, k = blockIdx.y;
    const size_t Et = (size_t)g.ntp * 256;
    const size_t per_k = Et + 2 * (size_t)p + 3;
    const size_t e = (size_t)blockIdx.x * kWave + threadIdx.x % kWave;
    double v = 0.0;
    if (e < Et)
        v = split_sum(tiles + (size_t)k * S * Et + e, Et, S);
    else if (e < Et + 2 * (size_t)p)
        v = split_sum(vec + (size_t)k * S * 2 * p + (e - Et), 2 * (size_t)p, S);
    else if (e < per_k)
        v = split_sum(scal + (size_t)k * S * 3 + (e - Et - 2 * p), 3, S);
    v = finish_combine(v, red);
    if (threadIdx.x >= kWave || e >= per_k) return;
    if (e < Et) {
        const int te = (int)(e % 256);
        const int tp = (int)(e / 256);
        int ti, tj;
        tile_pair_decode(tp, g.T, ti, tj);
        const int ei = te / 16, ej = te % 16;
        if (ti == tj && ei > ej) return;
        const int i = ti * 16 + ei, j = tj * 16 + ej;
        if (i >= p || j >= p) return;
        double *G = Gk + (size_t)k * p * p;
        G[(size_t)i * p + j] += v;
        if (i != j) G[(size_t)j * p + i] += v;
    } else if (e < Et + p) {
        bk[(size_t)k * p + (e - Et)] += v;
    } else if (e < Et + 2 * (size_t)p) {
        csk[(size_t)k * p + (e - Et - p)] += v;
    } else if (e == Et + 2 * (size_t)p) {
        yyk[k] += v;
    } else if (e == Et + 2 * (size_t)p + 1) {
        nk[k] += (int64_t)v;
    } else {
        ysk[k] += v;
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
    g.pa = p;
    g.tile = 16;
    g.T = (p + 15) / 16;
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

template <typename XT>
static int launch_f64_t(const GramGeom &g, bool list, bool vec, const XT *X, int64_t n, int64_t ldx,
                        const double *y, const RowSource &rs, double *part, double *pvec, double *pscal,
                        hipStream_t s, const CsrRows<XT> *csr = nullptr, const double *wts = nullptr)
{
    const int npanels = (g.nsb == 1) ? 1 : 2;
    const size_t lds = std::max((size_t)npanels * kRows * panel_pitch<XT>() * sizeof(XT) + kRows * sizeof(double),
                                (size_t)(16 * kPanelCols + 16) * sizeof(double));
    const void *kern;
    if (wts) kern = vec ? (const void *)gram_f64_kernel<XT, false, true, false, true>
                        : (const void *)gram_f64_kernel<XT, false, false, false, true>;
    else if (csr) kern = list ? (const void *)gram_f64_kernel<XT, true, false, true, false>
                              : (const void *)gram_f64_kernel<XT, false, false, true, false>;
    else if (list) kern = vec ? (const void *)gram_f64_kernel<XT, true, true, false, false>
                              : (const void *)gram_f64_kernel<XT, true, false, false, false>;
    else kern = vec ? (const void *)gram_f64_kernel<XT, false, true, false, false>
                    : (const void *)gram_f64_kernel<XT, false, false, false, false>;
    const unsigned blocks = (unsigned)(g.K * g.nsplit * g.npsb);
    OEM_HIP_CHECK(hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    CsrRows<XT> cr = csr ? *csr : CsrRows<XT>{nullptr, nullptr, nullptr, 0};
    void *args[] = {(void *)&X, (void *)&n, (void *)&ldx, (void *)&y, (void *)&g, (void *)&rs,
                    (void *)&part, (void *)&pvec, (void *)&pscal, (void *)&cr, (void *)&wts};
    OEM_HIP_CHECK(hipLaunchKernel(kern, dim3(blocks), dim3(kGramThreads), args, lds, s));
    return OEM_OK;
}

// Sparse rows handed to a pass (values of the handle's element type).
struct CsrIn {
    const int64_t *rowptr;
    const int32_t *col;
    const void *val;
    int64_t nnz;
};

static int launch_gram_any(oem_gram_s *h, const void *X, int64_t n, int64_t ldx, const double *y,
                           int64_t row_offset, const uint8_t *foldid, hipStream_t s, GramWork *ws,
                           const CsrIn *csr, const double *wts = nullptr);

static size_t f64_partial_bytes(const GramGeom &g)
{
    const size_t parts = (size_t)g.K * g.nsplit;
    return (parts * ((size_t)g.ntp * 256 + 2 * (size_t)g.p + 3) + 8) * sizeof(double);
}

size_t gram_work_bytes(const oem_gram_s *h, int64_t n)
{
    if (!gram_pass_fp64(h->prec, n)) {
        // same row-list plan as the BF16 pass (its geometry differs only in tiles)
        return gram_bf16_work_bytes(h->prec, h->p, h->K, n);
    }
    const GramGeom g = plan_f64(h->prec, h->p, h->K, n);
    return gram_carve_size(row_list_bytes(g, n)) + gram_carve_size(f64_partial_bytes(g));
}

int launch_gram(oem_gram_s *h, const void *X, int64_t n, int64_t ldx, const double *y,
                int64_t row_offset, const uint8_t *foldid, hipStream_t s, GramWork *ws)
{
    return launch_gram_any(h, X, n, ldx, y, row_offset, foldid, s, ws, nullptr);
}

int launch_gram_csr(oem_gram_s *h, const int64_t *rowptr, const int32_t *col, const void *val, int64_t nnz,
                    int64_t n, const double *y, int64_t row_offset, const uint8_t *foldid, hipStream_t s)
{
    if (h->prec != OEM_FP64) return fail(OEM_E_INVAL, "sparse rows take the FP64 Gram form");
    const CsrIn in{rowptr, col, val, nnz};
    return launch_gram_any(h, val, n, h->p, y, row_offset, foldid, s, nullptr, &in);
}

int launch_gram_weighted(oem_gram_s *h, const void *X, int64_t n, int64_t ldx, const double *y,
                         const double *wts, hipStream_t s)
{
    if (h->prec != OEM_FP64 || h->K != 1) return fail(OEM_E_STATE, "the weighted Gram pass takes the FP64 form, one fold");
    return launch_gram_any(h, X, n, ldx, y, 0, nullptr, s, nullptr, nullptr, wts);
}

static int launch_gram_any(oem_gram_s *h, const void *X, int64_t n, int64_t ldx, const double *y,
                           int64_t row_offset, const uint8_t *foldid, hipStream_t s, GramWork *ws,
                           const CsrIn *csr, const double *wts)
{
    if (!gram_pass_fp64(h->prec, n)) return launch_gram_bf16(h, X, n, ldx, y, row_offset, foldid, s, ws);
    const GramGeom g = plan_f64(h->prec, h->p, h->K, n);
    RowSource rs;
    int rc = build_row_lists(h, g, n, row_offset, foldid, rs, s, ws);
    if (rc) return rc;
    const size_t K = g.K, S = g.nsplit;
    const size_t Et = (size_t)g.ntp * 256;
    const size_t parts = K * S;
    void *pbuf = nullptr;
    rc = gram_buffer(h->partial, ws, f64_partial_bytes(g), &pbuf);
    if (rc) return rc;
    double *part = static_cast<double *>(pbuf);
    double *pvec = part + parts * Et;
    double *pscal = pvec + parts * 2 * g.p;
    const bool list = g.K > 1;
    if (h->xdt == OEM_X_F32) {
        const float *Xf = static_cast<const float *>(X);
        const bool vec = (reinterpret_cast<uintptr_t>(Xf) & 3) == 0;
        const CsrRows<float> cr = csr ? CsrRows<float>{csr->rowptr, csr->col, static_cast<const float *>(csr->val), csr->nnz}
                                      : CsrRows<float>{};
        rc = launch_f64_t<float>(g, list, vec, Xf, n, ldx, y, rs, part, pvec, pscal, s, csr ? &cr : nullptr, wts);
    } else {
        const double *Xd = static_cast<const double *>(X);
        const bool vec = (reinterpret_cast<uintptr_t>(Xd) & 7) == 0;
        const CsrRows<double> cr = csr ? CsrRows<double>{csr->rowptr, csr->col, static_cast<const double *>(csr->val), csr->nnz}
                                       : CsrRows<double>{};
        rc = launch_f64_t<double>(g, list, vec, Xd, n, ldx, y, rs, part, pvec, pscal, s, csr ? &cr : nullptr, wts);
    }
    if (rc) return rc;
    const size_t per_k = Et + 2 * (size_t)g.p + 3;
    const dim3 fgrid((unsigned)((per_k + kWave - 1) / kWave), (unsigned)K);
    hipLaunchKernelGGL(gram_f64_finish_kernel, fgrid, dim3(kFinishThreads), 0, s, g, part, pvec, pscal,
                       h->Gk.as<double>(), h->bk.as<double>(), h->yyk.as<double>(), h->nk.as<int64_t>(),
                       h->csk.as<double>(), h->ysk.as<double>());
    OEM_HIP_CHECK(hipGetLastError());
    return OEM_OK;
}

} // namespace oem
