// Streaming Gram pass (Section 3: per-fold X_k^T X_k and X_k^T y_k in one
// pass over the rows) for gfx950.
//
// FP64 form: the augmented matrix [X y] is staged through LDS in row chunks
// (FP32 X widened exactly) and multiplied on the FP64 matrix cores
// (v_mfma_f64_16x16x4f64).  The upper triangle of [X y]^T [X y] holds
// X^T X, X^T y (column p) and y^T y (corner), so one contraction gives every
// statistic.
//
// Work decomposition: the upper triangle of 16x16 tiles is cut into
// super-blocks of W x W tiles; a workgroup owns one (fold, row split,
// super-block pair).  With several folds a workgroup hashes the rows of its
// split and gathers only those of its fold, so every row is fetched once per
// super-block pair.  Workgroups sharing a row split are numbered so that the
// hardware's round-robin dispatch places them on one XCD, where they share
// that XCD's L2.  Each workgroup writes its partial tiles; a second kernel
// adds the partials of all splits in a fixed order (deterministic, no
// floating-point atomics).
#include <algorithm>

#include "oem_internal.h"

namespace oem {

typedef double d4_t __attribute__((ext_vector_type(4)));

constexpr int kGramThreads = 256;
constexpr int kGramWaves = kGramThreads / kWave;
constexpr int kMaxW = 8;                                   // tiles per super-block side
constexpr int kMaxSlots = (kMaxW * kMaxW + kGramWaves - 1) / kGramWaves;  // tile pairs per wave
constexpr int kRing = 512;                                 // gathered-row ring (power of 2)

// LDS row pitch (doubles) of a staged panel: a multiple of 16 that is odd in
// units of 16, so the four 16-lane row groups of an MFMA operand read fall on
// disjoint bank halves.
__host__ __device__ inline int panel_pitch(int W)
{
    int w = W * 16;
    return (W % 2 == 0) ? w + 16 : w;
}

// Logical block index: consecutive logical ids land on the same XCD under
// round-robin dispatch of hardware ids over the 8 XCDs.
__device__ inline int xcd_logical(int bid, int nb)
{
    const int nx = 8;
    int per = (nb + nx - 1) / nx;
    int full = (nb % nx == 0) ? nx : nb % nx;
    int x = bid % nx, local = bid / nx;
    if (x < full) return x * per + local;
    return full * per + (x - full) * (per - 1) + local;
}

__host__ __device__ inline int tile_pair_index(int ti, int tj, int T)
{
    return ti * T - (ti * (ti - 1)) / 2 + (tj - ti);
}

template <typename XT>
__device__ inline double load_aug(const XT *__restrict__ X, const double *__restrict__ y,
                                  int64_t row, int64_t ldx, int col, int p)
{
    if (col < p) return (double)X[row * ldx + col];
    if (col == p) return y[row];
    return 0.0;
}

// Stage rows rowid[0..nr) (absolute row indices; nr <= rk) of columns
// [c0, c0 + width) of [X y] into an LDS panel; rows nr..rk-1 are zero.
template <typename XT>
__device__ inline void stage_panel(double *panel, int pitch, int rk, int width, int c0,
                                   const XT *__restrict__ X, const double *__restrict__ y,
                                   int64_t ldx, int p, const int64_t *rows, int nr)
{
    const int total = rk * width;
    for (int e = threadIdx.x; e < total; e += kGramThreads) {
        int r = e / width, c = e - r * width;
        double v = 0.0;
        if (r < nr) v = load_aug(X, y, rows[r], ldx, c0 + c, p);
        panel[r * pitch + c] = v;
    }
}

template <typename XT>
__global__ __launch_bounds__(kGramThreads) void gram_f64_kernel(
    const XT *__restrict__ X, int64_t n, int64_t ldx, const double *__restrict__ y,
    int64_t row_offset, const uint8_t *__restrict__ foldid, uint64_t seed, GramGeom g,
    double *__restrict__ partial, int64_t *__restrict__ partial_n)
{
    extern __shared__ double smem[];
    const int lane = threadIdx.x % kWave;
    const int wave = threadIdx.x / kWave;

    const int L = xcd_logical(blockIdx.x, gridDim.x);
    const int q = L % g.npsb;
    const int rest = L / g.npsb;
    const int s = rest % g.nsplit;
    const int k = rest / g.nsplit;

    int I = 0, J = 0;
    {
        int qq = q;
        for (I = 0; I < g.nsb; ++I) {
            int cnt = g.nsb - I;
            if (qq < cnt) { J = I + qq; break; }
            qq -= cnt;
        }
    }
    const int Wi = min(g.W, g.T - I * g.W);
    const int Wj = min(g.W, g.T - J * g.W);
    const bool diag = (I == J);
    const int pitch = panel_pitch(g.W);

    double *A = smem;
    double *B = diag ? A : smem + g.rk * pitch;
    int64_t *ring = reinterpret_cast<int64_t *>(smem + 2 * g.rk * pitch);
    int64_t *chunk_rows = ring + kRing;                    // rk entries
    int *scan = reinterpret_cast<int *>(chunk_rows + g.rk); // kGramWaves + 1

    // this wave's tile pairs within the super-block pair
    const int npairs = diag ? Wi * (Wi + 1) / 2 : Wi * Wj;
    int ta[kMaxSlots], tb[kMaxSlots];
#pragma unroll
    for (int t = 0; t < kMaxSlots; ++t) {
        int m = wave + kGramWaves * t;
        int a = 0, b = 0;
        if (m < npairs) {
            if (diag) {
                int mm = m;
                for (a = 0; a < Wi; ++a) {
                    int cnt = Wi - a;
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

    const int64_t r0 = (int64_t)s * g.rows_per_split;
    const int64_t r1 = min(n, r0 + g.rows_per_split);
    const int colA = I * g.W * 16, colB = J * g.W * 16;
    const int widthA = Wi * 16, widthB = Wj * 16;

    auto mma_chunk = [&]() {
        for (int kk = 0; kk < g.rk / 4; ++kk) {
            const int row = 4 * kk + lane / 16;
#pragma unroll
            for (int t = 0; t < kMaxSlots; ++t) {
                if (t < nslots) {
                    double a = A[row * pitch + ta[t] * 16 + (lane % 16)];
                    double b = B[row * pitch + tb[t] * 16 + (lane % 16)];
                    acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[t], 0, 0, 0);
                }
            }
        }
    };

    auto process_chunk = [&](const int64_t *rows, int nr) {
        stage_panel(A, pitch, g.rk, widthA, colA, X, y, ldx, g.p, rows, nr);
        if (!diag) stage_panel(B, pitch, g.rk, widthB, colB, X, y, ldx, g.p, rows, nr);
        __syncthreads();
        mma_chunk();
        __syncthreads();
    };

    int64_t nmine = 0;
    if (g.K == 1) {
        for (int64_t c0 = r0; c0 < r1; c0 += g.rk) {
            int nr = (int)min<int64_t>(g.rk, r1 - c0);
            if (threadIdx.x < g.rk) chunk_rows[threadIdx.x] = c0 + threadIdx.x;
            __syncthreads();
            process_chunk(chunk_rows, nr);
            nmine += nr;
        }
    } else {
        // ordered gather of the split's rows that belong to fold k
        int head = 0, have = 0;
        for (int64_t b0 = r0; b0 < r1; b0 += kGramThreads) {
            const int64_t row = b0 + threadIdx.x;
            int mine = 0;
            if (row < r1) {
                uint32_t f = foldid ? (uint32_t)foldid[row]
                                    : fold_hash(seed, row_offset + row, (uint32_t)g.K);
                mine = (f == (uint32_t)k);
            }
            const uint64_t ball = __ballot(mine);
            const int before = __popcll(ball & ((1ull << lane) - 1ull));
            if (lane == 0) scan[wave] = __popcll(ball);
            __syncthreads();
            int off = 0, tot = 0;
            for (int w = 0; w < kGramWaves; ++w) {
                if (w < wave) off += scan[w];
                tot += scan[w];
            }
            if (mine) ring[(head + have + off + before) & (kRing - 1)] = row;
            __syncthreads();
            have += tot;
            while (have >= g.rk) {
                if (threadIdx.x < g.rk) chunk_rows[threadIdx.x] = ring[(head + threadIdx.x) & (kRing - 1)];
                __syncthreads();
                process_chunk(chunk_rows, g.rk);
                head = (head + g.rk) & (kRing - 1);
                have -= g.rk;
                nmine += g.rk;
            }
        }
        if (have > 0) {
            if (threadIdx.x < have) chunk_rows[threadIdx.x] = ring[(head + threadIdx.x) & (kRing - 1)];
            __syncthreads();
            process_chunk(chunk_rows, have);
            nmine += have;
        }
    }

    // epilogue: v_mfma_f64_16x16x4f64 leaves D[4 r + lane / 16][lane % 16] in
    // element r of lane's accumulator.
    const size_t base = ((size_t)k * g.nsplit + s) * (size_t)g.ntp;
#pragma unroll
    for (int t = 0; t < kMaxSlots; ++t) {
        if (t < nslots) {
            const int ti = I * g.W + ta[t], tj = J * g.W + tb[t];
            double *dst = partial + (base + tile_pair_index(ti, tj, g.T)) * 256;
#pragma unroll
            for (int r = 0; r < 4; ++r) dst[(4 * r + lane / 16) * 16 + (lane % 16)] = acc[t][r];
        }
    }
    if (q == 0 && threadIdx.x == 0) partial_n[(size_t)k * g.nsplit + s] = nmine;
}

// Sum the partials of every split in split order and add them to the running
// per-fold statistics; the upper triangle is mirrored so G stays exactly
// symmetric.
__global__ void gram_reduce_kernel(GramGeom g, const double *__restrict__ partial,
                                   const int64_t *__restrict__ partial_n, double *__restrict__ Gk,
                                   double *__restrict__ bk, double *__restrict__ yyk,
                                   int64_t *__restrict__ nk)
{
    const size_t total = (size_t)g.K * g.ntp * 256;
    const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx < (size_t)g.K) {
        int64_t c = 0;
        for (int s = 0; s < g.nsplit; ++s) c += partial_n[idx * g.nsplit + s];
        nk[idx] += c;
    }
    if (idx >= total) return;
    const int e = (int)(idx % 256);
    const int tp = (int)((idx / 256) % g.ntp);
    const int k = (int)(idx / ((size_t)256 * g.ntp));
    int ti = 0, tj = 0;
    {
        int t = tp;
        for (ti = 0; ti < g.T; ++ti) {
            int cnt = g.T - ti;
            if (t < cnt) { tj = ti + t; break; }
            t -= cnt;
        }
    }
    const int ei = e / 16, ej = e % 16;
    if (ti == tj && ei > ej) return;
    const int i = ti * 16 + ei, j = tj * 16 + ej;
    if (i > g.p || j > g.p) return;
    double sum = 0.0;
    const size_t stride = (size_t)g.ntp * 256;
    const double *src = partial + ((size_t)k * g.nsplit) * stride + (size_t)tp * 256 + e;
    for (int s = 0; s < g.nsplit; ++s) sum += src[(size_t)s * stride];
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

static GramGeom plan_f64(int p, int K, int64_t n)
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
    g.rk = 32;
    // enough workgroups to fill 256 CUs twice, but at least 256 rows per fold
    // in every split
    const int target = 512;
    int64_t ns = (target + (int64_t)K * g.npsb - 1) / ((int64_t)K * g.npsb);
    int64_t max_ns = std::max<int64_t>(1, n / (256 * (int64_t)K));
    ns = std::max<int64_t>(1, std::min(ns, max_ns));
    g.nsplit = (int)ns;
    g.rows_per_split = (n + ns - 1) / ns;
    return g;
}

static size_t gram_lds_bytes(const GramGeom &g)
{
    return (size_t)2 * g.rk * panel_pitch(g.W) * sizeof(double) + (size_t)kRing * sizeof(int64_t) +
           (size_t)g.rk * sizeof(int64_t) + (kGramWaves + 1) * sizeof(int);
}

int launch_gram(oem_gram_s *h, const void *X, int64_t n, int64_t ldx, const double *y,
                int64_t row_offset, const uint8_t *foldid, hipStream_t s)
{
    if (h->prec != OEM_FP64)
        return fail(OEM_E_INVAL, "this build computes the Gram in FP64 only");
    GramGeom g = plan_f64(h->p, h->K, n);
    const size_t npart = (size_t)g.K * g.nsplit * g.ntp * 256;
    int rc = h->partial.ensure(npart * sizeof(double));
    if (rc) return rc;
    rc = h->partial_n.ensure((size_t)g.K * g.nsplit * sizeof(int64_t));
    if (rc) return rc;
    const size_t lds = gram_lds_bytes(g);
    const int blocks = g.K * g.nsplit * g.npsb;
    if (lds > 64 * 1024) {
        OEM_HIP_CHECK(hipFuncSetAttribute((const void *)gram_f64_kernel<float>,
                                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
        OEM_HIP_CHECK(hipFuncSetAttribute((const void *)gram_f64_kernel<double>,
                                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    }
    if (h->xdt == OEM_X_F32) {
        hipLaunchKernelGGL(gram_f64_kernel<float>, dim3(blocks), dim3(kGramThreads), lds, s,
                           static_cast<const float *>(X), n, ldx, y, row_offset, foldid, h->seed,
                           g, h->partial.as<double>(), h->partial_n.as<int64_t>());
    } else {
        hipLaunchKernelGGL(gram_f64_kernel<double>, dim3(blocks), dim3(kGramThreads), lds, s,
                           static_cast<const double *>(X), n, ldx, y, row_offset, foldid, h->seed,
                           g, h->partial.as<double>(), h->partial_n.as<int64_t>());
    }
    OEM_HIP_CHECK(hipGetLastError());
    const size_t total = (size_t)g.K * g.ntp * 256;
    const int rblocks = (int)((total + 255) / 256);
    hipLaunchKernelGGL(gram_reduce_kernel, dim3(rblocks), dim3(256), 0, s, g,
                       h->partial.as<double>(), h->partial_n.as<int64_t>(), h->Gk.as<double>(),
                       h->bk.as<double>(), h->yyk.as<double>(), h->nk.as<int64_t>());
    OEM_HIP_CHECK(hipGetLastError());
    return OEM_OK;
}

} // namespace oem
