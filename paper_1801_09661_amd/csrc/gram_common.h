// Pieces shared by the Gram kernels: block numbering, row lists per
// (fold, split), and the fixed-order two-stage reduction of partial sums.
#pragma once

#include <algorithm>

#include "oem_internal.h"

namespace oem {

// Logical block index: consecutive logical ids land on the same XCD under
// round-robin dispatch of hardware block ids over the 8 XCDs, so blocks that
// read the same rows share that XCD's L2.
__device__ inline int xcd_logical(int bid, int nb)
{
    const int nx = 8;
    int per = (nb + nx - 1) / nx;
    int full = (nb % nx == 0) ? nx : nb % nx;
    int x = bid % nx, local = bid / nx;
    if (x < full) return x * per + local;
    return full * per + (x - full) * (per - 1) + local;
}

// Row-major numbering of the upper triangle of T x T tiles.
__host__ __device__ inline int tile_pair_index(int ti, int tj, int T)
{
    return ti * T - (ti * (ti - 1)) / 2 + (tj - ti);
}

__device__ inline void tile_pair_decode(int tp, int T, int &ti, int &tj)
{
    int t = tp;
    for (ti = 0; ti < T; ++ti) {
        const int cnt = T - ti;
        if (t < cnt) {
            tj = ti + t;
            return;
        }
        t -= cnt;
    }
}

// (I, J), I <= J, of super-block pair q in row-major upper-triangle order.
__device__ inline void sb_pair_decode(int q, int nsb, int &I, int &J)
{
    int qq = q;
    for (I = 0; I < nsb; ++I) {
        const int cnt = nsb - I;
        if (qq < cnt) {
            J = I + qq;
            return;
        }
        qq -= cnt;
    }
}

// Rows a workgroup streams: with one fold, the contiguous rows of its split;
// with several folds, the ordered list of its split's rows in its fold.
struct RowSource {
    const int32_t *list;     // K x (rows), segment (k, s) at off[k * S + s]
    const int64_t *off;      // K * S
    const int32_t *cnt;      // K * S
};

__device__ inline void rows_of(const GramGeom &g, const RowSource &rs, int64_t n, int k, int s,
                               int64_t &first, int64_t &count, const int32_t *&list)
{
    if (g.K == 1) {
        first = (int64_t)s * g.rows_per_split;
        const int64_t last = min(n, first + g.rows_per_split);
        count = last > first ? last - first : 0;
        list = nullptr;
    } else {
        const size_t i = (size_t)k * g.nsplit + s;
        first = 0;
        count = rs.cnt[i];
        list = rs.list + rs.off[i];
    }
}

__device__ inline int64_t row_at(int64_t first, const int32_t *list, int64_t i)
{
    return list ? (int64_t)list[i] : first + i;
}

// Columns a Gram loader thread reads for its group of four columns
// col .. col + 3 of a row of p elements.  vec: one 16-byte load of columns
// first .. first + 3 (the group lies inside the row, or lies wholly past its
// end and p >= 4, so columns 0..3 exist and are read instead); otherwise
// each column is read on its own, clamped to p - 1.  Either way every index
// read is below p.
struct GramColPlan {
    bool vec;
    int first;
};

__host__ __device__ inline GramColPlan gram_col_plan(bool vec_ok, int col, int p)
{
    GramColPlan c;
    c.vec = vec_ok && (col + 3 < p || (col >= p && p >= 4));
    c.first = (col + 3 < p) ? col : 0;
    return c;
}

__host__ __device__ inline int gram_col_read(const GramColPlan &c, int col, int j, int p)
{
    return c.vec ? c.first + j : (col + j < p - 1 ? col + j : p - 1);
}

// ---- host-side launchers (gram_common.hip) ----
// Target number of workgroups of a Gram pass (about two per CU by default;
// oem_gram_autotune may pick another for a shape).
constexpr int kGramDefaultTarget = 512;
// The split-BF16 form forms the products of a pass over fewer rows than this
// in FP64: the rounding errors of its BF16 parts (about 2^-17 relative per
// product, zero-mean) average over the rows of the pass, and below this many
// rows they move coefficients by more than 1e-6 relative (up to 5e-6 at
// 3600 rows, measured against the FP64 form), while the FP64 pass of so few
// rows is cheap.
constexpr int64_t kSplitMinRows = 32768;
// Whether a pass of n rows of this handle runs on the FP64 kernels.
inline bool gram_pass_fp64(int prec, int64_t n)
{
    return prec == OEM_FP64 || (prec == OEM_SPLIT_BF16 && n < kSplitMinRows);
}
int gram_target(int prec, int K, int p, int64_t n);
void gram_set_target(int prec, int K, int p, int64_t n, int target);
// Build per-(fold, split) ordered row lists for rows 0..n-1.
int build_row_lists(oem_gram_s *h, const GramGeom &g, int64_t n, int64_t row_offset,
                    const uint8_t *foldid, RowSource &rs, hipStream_t s, GramWork *ws);
// Bytes of those row lists (0 with one fold).
size_t row_list_bytes(const GramGeom &g, int64_t n);
// A buffer of `bytes` for one pass: carved (256-byte aligned) from ws when it
// has a base, else the handle's buffer `own`, grown as needed.
int gram_buffer(DevBuf &own, GramWork *ws, size_t bytes, void **out);
// Rounds a carved piece up to the carving alignment.
inline size_t gram_carve_size(size_t bytes) { return (bytes + 255) & ~size_t(255); }
// Partial-sum bytes of the BF16 forms' pass (gram_bf16.hip).
size_t gram_bf16_work_bytes(int prec, int p, int K, int64_t n);

// ---- split sums (device) ----
// Workgroups of kFinishThreads threads finish a Gram pass: each owns 64
// consecutive statistics of one fold; thread group h (threadIdx.x / 64) sums
// the splits s = h, h + 4, h + 8, ... of one statistic with four interleaved
// accumulators, and finish_combine adds the four groups' sums.  Every step has
// a fixed order, so the result is deterministic.
constexpr int kFinishThreads = 256;

template <typename T>
__device__ inline double split_sum(const T *__restrict__ base, size_t stride, int S)
{
    const int h = threadIdx.x / kWave;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    int s = h;
    // eight or four steps of the last loop at once, their 32 or 16 loads
    // issued together (one load round trip instead of eight or four; each
    // accumulator adds the same values in the same order)
    for (; s + 124 < S; s += 128) {
        double v[32];
#pragma unroll
        for (int j = 0; j < 32; ++j) v[j] = (double)base[(size_t)(s + 4 * j) * stride];
#pragma unroll
        for (int j = 0; j < 32; j += 4) {
            a0 += v[j];
            a1 += v[j + 1];
            a2 += v[j + 2];
            a3 += v[j + 3];
        }
    }
    for (; s + 60 < S; s += 64) {
        double v[16];
#pragma unroll
        for (int j = 0; j < 16; ++j) v[j] = (double)base[(size_t)(s + 4 * j) * stride];
#pragma unroll
        for (int j = 0; j < 16; j += 4) {
            a0 += v[j];
            a1 += v[j + 1];
            a2 += v[j + 2];
            a3 += v[j + 3];
        }
    }
    for (; s + 12 < S; s += 16) {
        a0 += (double)base[(size_t)s * stride];
        a1 += (double)base[(size_t)(s + 4) * stride];
        a2 += (double)base[(size_t)(s + 8) * stride];
        a3 += (double)base[(size_t)(s + 12) * stride];
    }
    for (; s < S; s += 4) a0 += (double)base[(size_t)s * stride];
    return (a0 + a1) + (a2 + a3);
}

// Sum of the four thread groups' values for lane `threadIdx.x % 64`, valid in
// group 0 (the others return 0).
__device__ inline double finish_combine(double v, double *red)
{
    const int lane = threadIdx.x % kWave, h = threadIdx.x / kWave;
    red[h * kWave + lane] = v;
    __syncthreads();
    if (h != 0) return 0.0;
    return (red[lane] + red[kWave + lane]) + (red[2 * kWave + lane] + red[3 * kWave + lane]);
}

} // namespace oem
