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
//   load   thread (q, rg) loads columns 4 q .. 4 q + 3 of 8 rows (16-byte
//          loads whatever the row pitch; a wave covers two 512-byte row
//          segments per load); the next chunk's loads are issued before the
//          current chunk's MFMAs, and rows past the end of the split are
//          read as copies of its last row and cleared before staging;
//   stage  the thread splits its values and writes each column's 8 rows as
//          one 16-byte LDS store into a column-major, slot-swizzled panel,
//          so one 16-byte read is an MFMA operand (8 consecutive rows of a
//          column) and neither access has bank conflicts;
//   mma    the waves form 2 pair groups x 2 k-groups: a pair group covers half
//          of the tile pairs, a k-group every other 16-row k-step, so each
//          wave reads a tile's operands once per k-step for several pairs;
//          the two k-groups' FP32 accumulators are added through LDS, in
//          wave order, when the workgroup finishes.  One launch covers the
//          diagonal and the off-diagonal super-block pairs.
// Partial tiles are FP32 and are summed over row splits in FP64 in a fixed
// order (deterministic, no floating-point atomics).
#include "gram_common.h"

namespace oem {

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x16_t __attribute__((ext_vector_type(16)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));
typedef float f32x2_t __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4_t __attribute__((ext_vector_type(4)));

constexpr int kBThreads = 256;
constexpr int kBTile = 32;                 // MFMA output tile
constexpr int kBMaxW = 4;                  // tiles per super-block side
constexpr int kBPanel = kBTile * kBMaxW;   // 128 columns per panel
constexpr int kBRows = 64;                 // rows per chunk: 4 MFMA k-steps of 16

// A staged panel is column-major: column c holds the chunk's 64 rows as
// eight 16-byte slots of 8 rows, slot s stored at position s ^ bswz(c).  The
// swizzle makes both access patterns conflict-free: a store covers columns
// 4 l + j of eight consecutive threads l (bits 2..4 of c vary), an operand
// read covers eight consecutive columns (bits 0..2 vary), and bswz is a
// bijection on both bit ranges.
__device__ inline int bswz(int c)
{
    return (c & 7) ^ ((c >> 3) & 3);
}

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

// Thread (q, rg) of a panel load: columns col .. col + 3 (col = base + 4 q)
// of the 8 rows `row`.  Columns at or past p are read from a valid column
// instead; they only feed tile entries that are discarded.
template <bool VEC>
__device__ inline void load_block(float (&x)[8][4], const float *const (&rp)[8], int p, int col)
{
    // 16-byte loads need only 4-byte alignment on gfx950 (column choice:
    // gram_col_plan).  rp: the 8 rows.
    const GramColPlan cp = gram_col_plan(VEC, col, p);
    if (cp.vec) {
        const int cv = cp.first;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const f32x4_t v = *reinterpret_cast<const f32x4_t *>(rp[e] + cv);
#pragma unroll
            for (int j = 0; j < 4; ++j) x[e][j] = v[j];
        }
    } else {
        int cj[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) cj[j] = gram_col_read(cp, col, j, p);
#pragma unroll
        for (int e = 0; e < 8; ++e)
#pragma unroll
            for (int j = 0; j < 4; ++j) x[e][j] = rp[e][cj[j]];
    }
}

template <bool SPLIT>
__device__ inline void stage_block(const float (&x)[8][4], __bf16 *hi, __bf16 *lo, int q, int rg)
{
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        // two rows per conversion: hi = bf16(v) of a pair in one packed
        // conversion, its FP32 value by bit operations, lo = bf16(v - hi)
        // of the pair in another (both round to nearest even)
        uint32_t hw[4], lw[4];
#pragma unroll
        for (int e = 0; e < 8; e += 2) {
            const float v0 = x[e][j], v1 = x[e + 1][j];
            const bf16x2_t h2 = __builtin_convertvector((f32x2_t){v0, v1}, bf16x2_t);
            const uint32_t hb = __builtin_bit_cast(uint32_t, h2);
            hw[e / 2] = hb;
            if (SPLIT) {
                const float h0 = __builtin_bit_cast(float, hb << 16);
                const float h1 = __builtin_bit_cast(float, hb & 0xffff0000u);
                const bf16x2_t l2 = __builtin_convertvector((f32x2_t){v0 - h0, v1 - h1}, bf16x2_t);
                lw[e / 2] = __builtin_bit_cast(uint32_t, l2);
            }
        }
        const int c = 4 * q + j;
        const int off = c * kBRows + 8 * (rg ^ bswz(c));
        *reinterpret_cast<u32x4_t *>(hi + off) = (u32x4_t){hw[0], hw[1], hw[2], hw[3]};
        if (SPLIT) *reinterpret_cast<u32x4_t *>(lo + off) = (u32x4_t){lw[0], lw[1], lw[2], lw[3]};
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

// The work of one workgroup: super-block pair (I, J) of row split s of fold
// k.  SPLIT: split-BF16 (else single BF16).  DIAG: a diagonal super-block
// (I = J; it also accumulates the FP64 diagonal, X^T y, y^T y, n and the
// column sums).  LIST: rows come from per-(fold, split) row lists (else the
// contiguous rows of the split).  VEC: 16-byte loads (X 4-byte aligned).
template <bool SPLIT, bool DIAG, bool LIST, bool VEC>
__device__ __forceinline__ void gram_bf16_block(
    const float *__restrict__ X, int64_t n, int64_t ldx, const double *__restrict__ y, const GramGeom &g,
    const RowSource &rs, float *__restrict__ partial, double *__restrict__ pvec, double *__restrict__ pscal,
    int k, int s, int I, int J, bool first_block)
{
    constexpr int NSLOT = DIAG ? 5 : 8;
    extern __shared__ char smem_raw[];
    const int lane = threadIdx.x % kWave;
    const int wave = threadIdx.x / kWave;
    const int q4 = threadIdx.x % 32, rg = threadIdx.x / 32;
    const int Wi = min(g.W, g.T - I * g.W);
    const int Wj = min(g.W, g.T - J * g.W);

    const int panel_elems = kBPanel * kBRows;
    // one staging buffer and one chunk of loads in flight (a second buffer
    // and a second chunk of loads were measured to gain nothing here)
    constexpr int NB = 1;
    constexpr int npan = DIAG ? 2 : 4;
    auto panels = [&](int b, __bf16 *&hA, __bf16 *&lA, __bf16 *&hB, __bf16 *&lB) {
        hA = reinterpret_cast<__bf16 *>(smem_raw) + (size_t)b * npan * panel_elems;
        lA = hA + panel_elems;
        hB = DIAG ? hA : lA + panel_elems;
        lB = DIAG ? lA : hB + panel_elems;
    };

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
    const int colA = I * g.W * kBTile + 4 * q4, colB = J * g.W * kBTile + 4 * q4;
    double sd[4] = {0.0, 0.0, 0.0, 0.0}, sxy[4] = {0.0, 0.0, 0.0, 0.0}, syy = 0.0;
    double sx[4] = {0.0, 0.0, 0.0, 0.0}, sy = 0.0;   // column sums and sum of y

    // the loads of the chunk in flight (one register set: NB = 1)
    float xa[NB][8][4], xb[NB][8][4];
    double yv[NB][8];
    int32_t nidx[8];      // row list entries of the next chunk to load (LIST)
    auto load_index = [&](int c) {
        if constexpr (LIST) {
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int64_t i = min((int64_t)c * kBRows + 8 * rg + e, count - 1);
                nidx[e] = list[i];
            }
        }
    };
    auto load_chunk = [&](int c, int r) {
        int64_t row[8];
        const float *rp[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            if constexpr (LIST) row[e] = nidx[e];
            else row[e] = first + min((int64_t)c * kBRows + 8 * rg + e, count - 1);
            rp[e] = X + row[e] * ldx;
        }
        load_block<VEC>(xa[r], rp, g.p, colA);
        if (!DIAG) load_block<VEC>(xb[r], rp, g.p, colB);
        if (DIAG) {
#pragma unroll
            for (int e = 0; e < 8; ++e) yv[r][e] = y[row[e]];
        }
    };
    // rows past the end of the split were read as copies of its last row
    auto clear_tail = [&](int c, int r) {
        const int64_t r0 = (int64_t)c * kBRows + 8 * rg;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            if (r0 + e >= count) {
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    xa[r][e][j] = 0.0f;
                    if (!DIAG) xb[r][e][j] = 0.0f;
                }
                if (DIAG) yv[r][e] = 0.0;
            }
        }
    };
    auto stage_chunk = [&](int r) {
        __bf16 *hA, *lA, *hB, *lB;
        panels(r, hA, lA, hB, lB);
        stage_block<SPLIT>(xa[r], hA, lA, q4, rg);
        if (!DIAG) stage_block<SPLIT>(xb[r], hB, lB, q4, rg);
        if (DIAG) {
#pragma unroll
            for (int e = 0; e < 8; ++e) {
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const double xd = (double)xa[r][e][j];
                    sd[j] += xd * xd;
                    sxy[j] += xd * yv[r][e];
                    sx[j] += xd;
                }
                syy += yv[r][e] * yv[r][e];
                sy += yv[r][e];
            }
        }
    };
    auto operand = [&](const __bf16 *panel, int tile, int ks) -> bf16x8_t {
        const int c = tile * kBTile + (lane % 32);
        const int slot = 2 * ks + lane / 32;
        return *reinterpret_cast<const bf16x8_t *>(panel + c * kBRows + 8 * (slot ^ bswz(c)));
    };
    auto mma_chunk = [&](int r) {
        __bf16 *hiA, *loA, *hiB, *loB;
        panels(r, hiA, loA, hiB, loB);
#pragma unroll
        for (int kh = 0; kh < kBRows / 32; ++kh) {
            const int ks = 2 * kh + ks0;
            if (DIAG) {
                // group 0 uses tiles 0..3, group 1 tiles 1..3
                // every pair of the group is formed (pairs past Wi read
                // staged columns of the panel and are not emitted), so the
                // accumulators are updated in place
                bf16x8_t h[kBMaxW], l[kBMaxW];
#pragma unroll
                for (int a = 0; a < kBMaxW; ++a) {
                    h[a] = operand(hiA, a, ks);
                    if (SPLIT) l[a] = operand(loA, a, ks);
                }
                if (pg == 0) {
#pragma unroll
                    for (int t = 0; t < 5; ++t)
                        acc[t] = mfma3<SPLIT>(acc[t], h[dg_a(0, t)], l[dg_a(0, t)], h[dg_b(0, t)], l[dg_b(0, t)]);
                } else {
#pragma unroll
                    for (int t = 0; t < 5; ++t)
                        acc[t] = mfma3<SPLIT>(acc[t], h[dg_a(1, t)], l[dg_a(1, t)], h[dg_b(1, t)], l[dg_b(1, t)]);
                }
            } else {
                bf16x8_t ah[2], al[2], bh[kBMaxW], bl[kBMaxW];
#pragma unroll
                for (int a = 0; a < 2; ++a) {
                    ah[a] = operand(hiA, 2 * pg + a, ks);
                    if (SPLIT) al[a] = operand(loA, 2 * pg + a, ks);
                }
#pragma unroll
                for (int b = 0; b < kBMaxW; ++b) {
                    bh[b] = operand(hiB, b, ks);
                    if (SPLIT) bl[b] = operand(loB, b, ks);
                }
#pragma unroll
                for (int a = 0; a < 2; ++a)
#pragma unroll
                    for (int b = 0; b < kBMaxW; ++b)
                        acc[4 * a + b] = mfma3<SPLIT>(acc[4 * a + b], ah[a], al[a], bh[b], bl[b]);
            }
        }
    };
    if (nchunks > 0) {
        load_index(0);
        load_chunk(0, 0);
        load_index(1);
    }
    for (int c = 0; c < nchunks; ++c) {
        if ((int64_t)(c + 1) * kBRows > count) clear_tail(c, 0);
        stage_chunk(0);
        __syncthreads();
        if (c + 1 < nchunks) {
            load_chunk(c + 1, 0);   // in flight during the products
            load_index(c + 2);
        }
        mma_chunk(0);
        __syncthreads();
    }

    // Sum the two k-groups' accumulators of each tile pair (in wave order)
    // and write the FP32 partial.  v_mfma_f32_32x32x16_bf16 leaves
    // D[8 (r / 4) + 4 (lane / 32) + r % 4][lane % 32] in element r.
    float *red = reinterpret_cast<float *>(smem_raw);   // 2 x 1024 floats
    const size_t part_id = (size_t)k * g.nsplit + s;
    auto put = [&](const f32x16_t &v, int slot) {
#pragma unroll
        for (int r = 0; r < 16; ++r)
            red[slot * 1024 + (8 * (r / 4) + 4 * (lane / 32) + (r % 4)) * kBTile + (lane % 32)] = v[r];
    };
    auto emit = [&](int ti, int tj) {
        __syncthreads();
        float *dst = partial + (part_id * g.ntp + tile_pair_index(ti, tj, g.T)) * (kBTile * kBTile);
        for (int e = threadIdx.x; e < 1024; e += kBThreads) dst[e] = red[e] + red[1024 + e];
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
                emit(I * g.W + a, J * g.W + b);
            }
        }
    }

    // FP64 diagonal, X^T y, column sums, y^T y, sum y: the 8 row groups of a
    // column are combined in order; pvec = [part][diag p | xy p | colsum p],
    // pscal = [part][yy, n, sum y]
    if (DIAG) {
        double *vred = reinterpret_cast<double *>(smem_raw);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            vred[rg * kBPanel + 4 * q4 + j] = sd[j];
            vred[8 * kBPanel + rg * kBPanel + 4 * q4 + j] = sxy[j];
            vred[16 * kBPanel + rg * kBPanel + 4 * q4 + j] = sx[j];
        }
        if (q4 == 0) {
            vred[24 * kBPanel + rg] = syy;
            vred[24 * kBPanel + 8 + rg] = sy;
        }
        __syncthreads();
        if (threadIdx.x < kBPanel) {
            const int col = I * g.W * kBTile + threadIdx.x;
            double d = 0.0, b = 0.0, c = 0.0;
            for (int r = 0; r < 8; ++r) {
                d += vred[r * kBPanel + threadIdx.x];
                b += vred[8 * kBPanel + r * kBPanel + threadIdx.x];
                c += vred[16 * kBPanel + r * kBPanel + threadIdx.x];
            }
            if (col < g.p) {
                pvec[part_id * 3 * g.p + col] = d;
                pvec[part_id * 3 * g.p + g.p + col] = b;
                pvec[part_id * 3 * g.p + 2 * g.p + col] = c;
            }
        }
        if (first_block && threadIdx.x == 0) {
            double t = 0.0, u = 0.0;
            for (int r = 0; r < 8; ++r) {
                t += vred[24 * kBPanel + r];
                u += vred[24 * kBPanel + 8 + r];
            }
            pscal[part_id * 3] = t;
            pscal[part_id * 3 + 1] = (double)count;
            pscal[part_id * 3 + 2] = u;
        }
    }
}

// One launch covers every (fold, row split, super-block pair).  The npsb
// pairs of one (fold, split) read the same rows; they take consecutive
// logical block numbers, which round-robin dispatch places on one XCD, so
// they run side by side and the rows come from HBM about once and from that
// XCD's L2 for the other pairs.  The diagonal pairs come first in each group.
// OFF: the geometry has off-diagonal pairs (p > 128); without them the kernel
// holds only the diagonal code and its smaller register set.
template <bool SPLIT, bool LIST, bool VEC, bool OFF>
__global__ __launch_bounds__(kBThreads, 2) void gram_bf16_kernel(
    const float *__restrict__ X, int64_t n, int64_t ldx, const double *__restrict__ y, GramGeom g,
    RowSource rs, float *__restrict__ partial, double *__restrict__ pvec, double *__restrict__ pscal)
{
    const int L = xcd_logical(blockIdx.x, gridDim.x);
    const int qq = L % g.npsb;
    const int rest = L / g.npsb;
    const int s = rest % g.nsplit;
    const int k = rest / g.nsplit;
    if (!OFF || qq < g.nsb) {
        gram_bf16_block<SPLIT, true, LIST, VEC>(X, n, ldx, y, g, rs, partial, pvec, pscal, k, s, qq, qq, qq == 0);
    } else if constexpr (OFF) {
        int t = qq - g.nsb, I = 0, J = 0;
        for (I = 0; I < g.nsb; ++I) {
            const int cnt = g.nsb - I - 1;
            if (t < cnt) { J = I + 1 + t; break; }
            t -= cnt;
        }
        gram_bf16_block<SPLIT, false, LIST, VEC>(X, n, ldx, y, g, rs, partial, pvec, pscal, k, s, I, J, false);
    }
}

// Finish the pass: sum each statistic over the row splits (fixed order) and
// add it into the running sums: off-diagonal tile entries (upper triangle,
// mirrored so G stays exactly symmetric), then the FP64 diagonal, X^T y and
// the column sums, then y^T y, n and sum y.  Grid (statistic blocks of 64,
// folds).
__global__ __launch_bounds__(kFinishThreads) void gram_bf16_finish_kernel(
    GramGeom g, const float *__restrict__ tiles, const double *__restrict__ vec,
    const double *__restrict__ scal, double *__restrict__ Gk, double *__restrict__ bk,
    double *__restrict__ yyk, int64_t *__restrict__ nk, double *__restrict__ csk,
    double *__restrict__ ysk)
{
    __shared__ double red[kFinishThreads];
    const int p = g.p, S = g.nsplit, k = blockIdx.y;
    const size_t tile = kBTile * kBTile;
    const size_t Et = (size_t)g.ntp * tile;
    const size_t per_k = Et + 3 * (size_t)p + 3;
    const size_t e = (size_t)blockIdx.x * kWave + threadIdx.x % kWave;
    double v = 0.0;
    if (e < Et)
        v = split_sum(tiles + (size_t)k * S * Et + e, Et, S);
    else if (e < Et + 3 * (size_t)p)
        v = split_sum(vec + (size_t)k * S * 3 * p + (e - Et), 3 * (size_t)p, S);
    else if (e < per_k)
        v = split_sum(scal + (size_t)k * S * 3 + (e - Et - 3 * p), 3, S);
    v = finish_combine(v, red);
    if (threadIdx.x >= kWave || e >= per_k) return;
    double *G = Gk + (size_t)k * p * p;
    if (e < Et) {
        const int te = (int)(e % tile);
        const int tp = (int)(e / tile);
        int ti, tj;
        tile_pair_decode(tp, g.T, ti, tj);
        const int ei = te / kBTile, ej = te % kBTile;
        if (ti == tj && ei >= ej) return;         // diagonal from FP64; lower half mirrored
        const int i = ti * kBTile + ei, j = tj * kBTile + ej;
        if (i >= p || j >= p) return;
        G[(size_t)i * p + j] += v;
        G[(size_t)j * p + i] += v;
    } else if (e < Et + 3 * (size_t)p) {
        const size_t c = e - Et;
        if (c < (size_t)p) G[c * p + c] += v;
        else if (c < 2 * (size_t)p) bk[(size_t)k * p + (c - p)] += v;
        else csk[(size_t)k * p + (c - 2 * p)] += v;
    } else if (e == Et + 3 * (size_t)p) {
        yyk[k] += v;
    } else if (e == Et + 3 * (size_t)p + 1) {
        nk[k] += (int64_t)v;
    } else {
        ysk[k] += v;
    }
}

static GramGeom plan_bf16(int prec, int p, int K, int64_t n)
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
    const int64_t target = gram_target(prec, K, p, n);
    int64_t ns = std::max<int64_t>(1, (target + (int64_t)K * g.npsb - 1) / ((int64_t)K * g.npsb));
    int64_t rps = (n + ns - 1) / ns;
    const int64_t quantum = (K == 1) ? kBRows : 4096;
    rps = std::max<int64_t>(quantum, (rps + quantum - 1) / quantum * quantum);
    g.rows_per_split = rps;
    g.nsplit = (int)std::max<int64_t>(1, (n + rps - 1) / rps);
    return g;
}

static size_t bf16_lds_bytes(bool off)
{
    // four panels with off-diagonal pairs (the diagonal ones use two), else
    // two; or the reduction areas, whichever is larger
    const size_t panels = (size_t)(off ? 4 : 2) * kBPanel * kBRows * sizeof(__bf16);
    const size_t red = std::max((size_t)2 * 1024 * sizeof(float), (size_t)(24 * kBPanel + 16) * sizeof(double));
    return std::max(panels, red);
}

template <bool SPLIT, bool OFF>
static const void *bf16_kernel(bool list, bool vec)
{
    if (list) return vec ? (const void *)gram_bf16_kernel<SPLIT, true, true, OFF>
                         : (const void *)gram_bf16_kernel<SPLIT, true, false, OFF>;
    return vec ? (const void *)gram_bf16_kernel<SPLIT, false, true, OFF>
               : (const void *)gram_bf16_kernel<SPLIT, false, false, OFF>;
}

template <bool SPLIT>
static int launch_bf16_t(const GramGeom &g, bool list, bool vec, unsigned blocks, const float *X,
                         int64_t n, int64_t ldx, const double *y, const RowSource &rs, float *part,
                         double *pvec, double *pscal, hipStream_t s)
{
    const void *kern = g.npsb > g.nsb ? bf16_kernel<SPLIT, true>(list, vec) : bf16_kernel<SPLIT, false>(list, vec);
    const size_t lds = bf16_lds_bytes(g.npsb > g.nsb);
    OEM_HIP_CHECK(hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    void *args[] = {(void *)&X, (void *)&n, (void *)&ldx, (void *)&y, (void *)&g, (void *)&rs,
                    (void *)&part, (void *)&pvec, (void *)&pscal};
    OEM_HIP_CHECK(hipLaunchKernel(kern, dim3(blocks), dim3(kBThreads), args, lds, s));
    return OEM_OK;
}

static size_t bf16_partial_bytes(const GramGeom &g)
{
    const size_t parts = (size_t)g.K * g.nsplit;
    const size_t Et = (size_t)g.ntp * kBTile * kBTile;
    return parts * Et * sizeof(float) + parts * (3 * (size_t)g.p + 3) * sizeof(double) + 64;
}

size_t gram_bf16_work_bytes(int prec, int p, int K, int64_t n)
{
    const GramGeom g = plan_bf16(prec, p, K, n);
    return gram_carve_size(row_list_bytes(g, n)) + gram_carve_size(bf16_partial_bytes(g));
}

int launch_gram_bf16(oem_gram_s *h, const void *Xv, int64_t n, int64_t ldx, const double *y,
                     int64_t row_offset, const uint8_t *foldid, hipStream_t s, GramWork *ws)
{
    if (h->xdt != OEM_X_F32) return fail(OEM_E_INVAL, "the BF16 Gram forms take FP32 X");
    const float *X = static_cast<const float *>(Xv);
    const GramGeom g = plan_bf16(h->prec, h->p, h->K, n);
    RowSource rs;
    int rc = build_row_lists(h, g, n, row_offset, foldid, rs, s, ws);
    if (rc) return rc;
    const size_t S = g.nsplit, K = g.K;
    const size_t Et = (size_t)g.ntp * kBTile * kBTile;
    const size_t parts = K * S;
    void *pbuf = nullptr;
    rc = gram_buffer(h->partial, ws, bf16_partial_bytes(g), &pbuf);
    if (rc) return rc;
    float *part = static_cast<float *>(pbuf);
    double *pvec = reinterpret_cast<double *>(part + parts * Et);
    double *pscal = pvec + parts * 3 * g.p;

    const bool split = (h->prec == OEM_SPLIT_BF16);
    const bool list = g.K > 1;
    const bool vec = (reinterpret_cast<uintptr_t>(X) & 3) == 0;
    const unsigned nb = (unsigned)(g.K * g.nsplit * g.npsb);
    rc = split ? launch_bf16_t<true>(g, list, vec, nb, X, n, ldx, y, rs, part, pvec, pscal, s)
               : launch_bf16_t<false>(g, list, vec, nb, X, n, ldx, y, rs, part, pvec, pscal, s);
    if (rc) return rc;
    const size_t per_k = Et + 3 * (size_t)g.p + 3;
    const dim3 fgrid((unsigned)((per_k + kWave - 1) / kWave), (unsigned)K);
    hipLaunchKernelGGL(gram_bf16_finish_kernel, fgrid, dim3(kFinishThreads), 0, s, g, part, pvec, pscal,
                       h->Gk.as<double>(), h->bk.as<double>(), h->yyk.as<double>(), h->nk.as<int64_t>(),
                       h->csk.as<double>(), h->ysk.as<double>());
    OEM_HIP_CHECK(hipGetLastError());
    return OEM_OK;
}

} // namespace oem
