// Row lists per (fold, split) and the fixed-order reduction of Gram partials.
//
// Rows are cut into blocks of kListBlock rows.  count: per block, the number
// of rows in each fold; scan: exclusive prefix over (fold, block) in fold-major
// order; scatter: each block writes its rows, in row order, into its fold's
// run.  The list of fold k is therefore the rows of fold k in ascending order,
// and a split (a whole number of blocks) owns a contiguous piece of it.
#include "gram_common.h"

#include <map>
#include <mutex>
#include <tuple>

namespace oem {

// ---------------------------------------------------------------- tuning
// Workgroup-count targets of the Gram pass chosen by oem_gram_autotune,
// keyed by (precision, folds > 1, p rounded up to 32, floor(log2 n)).
static std::mutex g_tune_mu;
static std::map<std::tuple<int, int, int, int>, int> g_tune;

static std::tuple<int, int, int, int> tune_key(int prec, int K, int p, int64_t n)
{
    int lg = 0;
    while (lg < 62 && (int64_t(1) << (lg + 1)) <= n) ++lg;
    return std::make_tuple(prec, K > 1 ? 1 : 0, (p + 31) / 32, lg);
}

int gram_target(int prec, int K, int p, int64_t n)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune.find(tune_key(prec, K, p, n));
    return it == g_tune.end() ? kGramDefaultTarget : it->second;
}

void gram_set_target(int prec, int K, int p, int64_t n, int target)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune[tune_key(prec, K, p, n)] = target;
}

constexpr int kListBlock = 4096;
constexpr int kListThreads = 256;
constexpr int kListWaves = kListThreads / kWave;
constexpr int kMaxFolds = 64;

__device__ inline uint32_t row_fold(int64_t row, int64_t row_offset, const uint8_t *foldid,
                                    uint64_t seed, int K)
{
    return foldid ? (uint32_t)foldid[row] : fold_hash(seed, row_offset + row, (uint32_t)K);
}

__global__ __launch_bounds__(kListThreads) void fold_count_kernel(int64_t n, int64_t row_offset,
                                                                  const uint8_t *__restrict__ foldid,
                                                                  uint64_t seed, int K, int nb,
                                                                  int32_t *__restrict__ counts)
{
    __shared__ int hist[kMaxFolds];
    const int b = blockIdx.x;
    for (int k = threadIdx.x; k < K; k += kListThreads) hist[k] = 0;
    __syncthreads();
    const int64_t r0 = (int64_t)b * kListBlock;
    const int64_t r1 = min(n, r0 + kListBlock);
    for (int64_t r = r0 + threadIdx.x; r < r1; r += kListThreads) {
        const uint32_t f = row_fold(r, row_offset, foldid, seed, K);
        if (f < (uint32_t)K) atomicAdd(&hist[f], 1);
    }
    __syncthreads();
    for (int k = threadIdx.x; k < K; k += kListThreads) counts[(size_t)k * nb + b] = hist[k];
}

// Exclusive prefix of counts (K x nb, fold-major) into off; one workgroup.
__global__ __launch_bounds__(kListThreads) void fold_scan_kernel(const int32_t *__restrict__ counts,
                                                                 int64_t total_entries,
                                                                 int64_t *__restrict__ off)
{
    __shared__ int64_t part[kListThreads];
    const int64_t per = (total_entries + kListThreads - 1) / kListThreads;
    const int64_t a = (int64_t)threadIdx.x * per;
    const int64_t e = min(total_entries, a + per);
    int64_t s = 0;
    for (int64_t i = a; i < e; ++i) s += counts[i];
    part[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t run = 0;
        for (int t = 0; t < kListThreads; ++t) {
            const int64_t v = part[t];
            part[t] = run;
            run += v;
        }
    }
    __syncthreads();
    int64_t run = part[threadIdx.x];
    for (int64_t i = a; i < e; ++i) {
        off[i] = run;
        run += counts[i];
    }
}

__global__ __launch_bounds__(kListThreads) void fold_scatter_kernel(
    int64_t n, int64_t row_offset, const uint8_t *__restrict__ foldid, uint64_t seed, int K, int nb,
    const int64_t *__restrict__ off, int32_t *__restrict__ list)
{
    __shared__ int wcount[kListWaves][kMaxFolds];
    __shared__ int64_t run[kMaxFolds];
    const int b = blockIdx.x;
    const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
    for (int k = threadIdx.x; k < K; k += kListThreads) run[k] = off[(size_t)k * nb + b];
    __syncthreads();
    const int64_t r0 = (int64_t)b * kListBlock;
    const int64_t r1 = min(n, r0 + kListBlock);
    const uint64_t below = (1ull << lane) - 1ull;
    for (int64_t base = r0; base < r1; base += kListThreads) {
        const int64_t r = base + threadIdx.x;
        const uint32_t f = (r < r1) ? row_fold(r, row_offset, foldid, seed, K) : 0xFFFFFFFFu;
        int rank = 0;
        for (int k = 0; k < K; ++k) {
            const uint64_t m = __ballot(f == (uint32_t)k);
            if (f == (uint32_t)k) rank = __popcll(m & below);
            if (lane == 0) wcount[wave][k] = __popcll(m);
        }
        __syncthreads();
        if (f < (uint32_t)K) {
            int64_t pos = run[f] + rank;
            for (int w = 0; w < wave; ++w) pos += wcount[w][f];
            list[pos] = (int32_t)r;
        }
        __syncthreads();
        for (int k = threadIdx.x; k < K; k += kListThreads) {
            int t = 0;
            for (int w = 0; w < kListWaves; ++w) t += wcount[w][k];
            run[k] += t;
        }
        __syncthreads();
    }
}

// Segment (k, s) = blocks [s * bps, (s + 1) * bps) of fold k's run.
__global__ void fold_segments_kernel(const int64_t *__restrict__ off,
                                     const int32_t *__restrict__ counts, int K, int nb, int S,
                                     int bps, int64_t *__restrict__ seg_off,
                                     int32_t *__restrict__ seg_cnt)
{
    const int64_t total = off[(size_t)K * nb - 1] + counts[(size_t)K * nb - 1];
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= K * S) return;
    const int k = i / S, s = i % S;
    const int b0 = s * bps, b1 = min(nb, (s + 1) * bps);
    const int64_t start = off[(size_t)k * nb + min(b0, nb - 1)];
    int64_t end;
    if (b1 < nb) end = off[(size_t)k * nb + b1];
    else end = (k + 1 < K) ? off[(size_t)(k + 1) * nb] : total;
    const bool empty = b0 >= nb;
    seg_off[i] = empty ? 0 : start;
    seg_cnt[i] = empty ? 0 : (int32_t)(end - start);
}

size_t row_list_bytes(const GramGeom &g, int64_t n)
{
    if (g.K == 1) return 0;
    const int nb = (int)((n + kListBlock - 1) / kListBlock);
    const size_t entries = (size_t)g.K * nb;
    const size_t segs = (size_t)g.K * g.nsplit;
    return n * sizeof(int32_t) + entries * (sizeof(int32_t) + sizeof(int64_t)) +
           segs * (sizeof(int64_t) + sizeof(int32_t)) + 64;
}

int gram_buffer(DevBuf &own, GramWork *ws, size_t bytes, void **out)
{
    if (!ws || !ws->base) {
        int rc = own.ensure(bytes);
        if (rc) return rc;
        *out = own.ptr;
        return OEM_OK;
    }
    const size_t need = ws->used + gram_carve_size(bytes);
    if (need > ws->bytes)
        return fail(OEM_E_INVAL, "the Gram pass needs " + std::to_string(need) +
                                     " bytes of workspace; the limit is " + std::to_string(ws->bytes));
    *out = ws->base + ws->used;
    ws->used = need;
    return OEM_OK;
}

int build_row_lists(oem_gram_s *h, const GramGeom &g, int64_t n, int64_t row_offset,
                    const uint8_t *foldid, RowSource &rs, hipStream_t s, GramWork *ws)
{
    rs = RowSource{nullptr, nullptr, nullptr};
    if (g.K == 1) return OEM_OK;
    if (g.K > kMaxFolds) return fail(OEM_E_INVAL, "at most 64 folds");
    if (g.rows_per_split % kListBlock != 0) return fail(OEM_E_STATE, "split is not a whole number of row blocks");
    const int nb = (int)((n + kListBlock - 1) / kListBlock);
    const int bps = (int)(g.rows_per_split / kListBlock);
    const size_t entries = (size_t)g.K * nb;
    const size_t segs = (size_t)g.K * g.nsplit;
    void *buf = nullptr;
    int rc = gram_buffer(h->rowlist, ws, row_list_bytes(g, n), &buf);
    if (rc) return rc;
    char *base = static_cast<char *>(buf);
    int64_t *off = reinterpret_cast<int64_t *>(base);
    int64_t *seg_off = off + entries;
    int32_t *counts = reinterpret_cast<int32_t *>(seg_off + segs);
    int32_t *seg_cnt = counts + entries;
    int32_t *list = seg_cnt + segs;
    hipLaunchKernelGGL(fold_count_kernel, dim3(nb), dim3(kListThreads), 0, s, n, row_offset, foldid,
                       h->seed, g.K, nb, counts);
    OEM_HIP_CHECK(hipGetLastError());
    hipLaunchKernelGGL(fold_scan_kernel, dim3(1), dim3(kListThreads), 0, s, counts, (int64_t)entries, off);
    OEM_HIP_CHECK(hipGetLastError());
    hipLaunchKernelGGL(fold_scatter_kernel, dim3(nb), dim3(kListThreads), 0, s, n, row_offset, foldid,
                       h->seed, g.K, nb, off, list);
    OEM_HIP_CHECK(hipGetLastError());
    hipLaunchKernelGGL(fold_segments_kernel, dim3((unsigned)((segs + 255) / 256)), dim3(256), 0, s, off,
                       counts, g.K, nb, g.nsplit, bps, seg_off, seg_cnt);
    OEM_HIP_CHECK(hipGetLastError());
    rs.list = list;
    rs.off = seg_off;
    rs.cnt = seg_cnt;
    return OEM_OK;
}

} // namespace oem

// Test hook (include/oem_debug.h): the four column indices the Gram loaders
// read for the group col .. col + 3 of a row of p elements.
extern "C" int oem_debug_gram_load_columns(int32_t p, int32_t col, int32_t vec_ok, int32_t *cols)
{
    if (p < 1 || col < 0 || !cols) return OEM_E_INVAL;
    const oem::GramColPlan c = oem::gram_col_plan(vec_ok != 0, col, p);
    for (int j = 0; j < 4; ++j) cols[j] = oem::gram_col_read(c, col, j, p);
    return c.vec ? 1 : 0;
}
