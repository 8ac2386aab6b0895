// Internal declarations shared by the HIP translation units of liboem.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/oem.h"

namespace oem {

constexpr int kWave = 64;

// ------------------------------------------------------------------ errors
void set_error(const std::string &msg);
int fail(int code, const std::string &msg);

#define OEM_HIP_CHECK(expr)                                                        \
    do {                                                                           \
        hipError_t e_ = (expr);                                                    \
        if (e_ != hipSuccess)                                                      \
            return ::oem::fail(OEM_E_HIP, std::string(#expr) + ": " +              \
                                              hipGetErrorString(e_));              \
    } while (0)

// ------------------------------------------------------------------ memory
// A pointer read from memory (a descriptor field) is generic to the
// compiler, so accesses through it become flat instructions, which also
// count against the LDS wait counter: every LDS wait then waits for the
// outstanding global loads as well.  gmem() marks such a pointer as global
// memory.
template <typename T> __device__ inline __attribute__((address_space(1))) T *gmem(T *p)
{
    return (__attribute__((address_space(1))) T *)p;
}

// ------------------------------------------------------------------ fold hash
// SplitMix64 (Steele, Lea & Flood 2014): the (i+1)-th output from state seed
// is mix64(seed + (i+1) * 0x9E3779B97F4A7C15).  The fold is the high word
// scaled to [0, K).
__host__ __device__ inline uint32_t fold_hash(uint64_t seed, int64_t row, uint32_t K)
{
    uint64_t z = seed + (uint64_t)(row + 1) * 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    z ^= z >> 31;
    return (uint32_t)(((z >> 32) * (uint64_t)K) >> 32);
}

// ------------------------------------------------------------------ penalties
// Penalties whose update works on whole groups (Section 2.2).
__host__ __device__ inline bool group_penalty(int kind)
{
    return kind == OEM_GRP_LASSO || kind == OEM_GRP_MCP || kind == OEM_GRP_SCAD || kind == OEM_SGL;
}

// ------------------------------------------------------------------ Gram geometry
// The Gram pass computes the upper triangle of the augmented Gram
// [X y]^T [X y] in square tiles.  Tiles are grouped into super-blocks of W
// tiles; one workgroup owns one (fold, row split, super-block pair).
struct GramGeom {
    int p;            // columns of X
    int pa;           // columns carried through the matrix cores (p + 1 in FP64: y appended)
    int tile;         // 16 (FP64 MFMA) or 32 (BF16 MFMA)
    int T;            // tiles per side
    int W;            // tiles per super-block side
    int nsb;          // super-blocks per side
    int npsb;         // super-block pairs (upper triangle)
    int ntp;          // tile pairs (upper triangle) = T (T + 1) / 2
    int K;            // folds
    int nsplit;       // row splits
    int64_t rows_per_split;
    int rk;           // rows per LDS stage
};

// ------------------------------------------------------------------ paths
// One warm-started lambda path: a (problem, penalty) pair.
struct PathDesc {
    const double *G;      // p x p standardised Gram (scaled by 1/n)
    const double *c;      // p
    const double *s;      // p column scales (beta = beta_std / s)
    const double *yyn;    // 1
    const double *d;      // 1
    const double *lambda; // L
    double *beta;         // L x p original scale
    double *beta_std;     // L x p standardised scale or null
    int32_t *iters;       // L or null
    double *kkt;          // L or null
    double *obj;          // L or null
    const int32_t *gstart;  // ngroups + 1 (group penalties)
    const int32_t *gidx;    // p
    const double *w;        // p or null
    const double *cg;       // ngroups
    int32_t p;
    int32_t L;
    int32_t kind;
    int32_t ngroups;
    double alpha;
    double gamma;
    double tau;           // sparse group lasso mixing
    double tol;
    int32_t maxit;
    // hand-over between the kernels of one path's launch chain: the first
    // lambda index the next kernel computes, and the standardised
    // coefficients of the lambda before it (p)
    int32_t *lstart;
    double *bws;
    // intercept (centred problems): means of the problem's rows, and the
    // output ybar - xbar^T beta per lambda (L), or null
    const double *xbar;
    const double *ybar;
    double *beta0;
    // warm start of the first lambda (standardised scale, p), or null for
    // beta = 0; paths with a warm start run on the general kernel
    const double *beta_init;
};

// ------------------------------------------------------------------ Lanczos jobs
// One problem of a batched Lanczos launch (d = lambda_1 (1 + 1e-10) of G).
struct LzJob {
    const double *G;     // p x p
    double *V;           // (mmax + 1) x p workspace for p > 128, else unused
    double *d;           // output
    int32_t *steps;      // output or null
    int p;
    int mmax;
};
// Step count written when the multi-workgroup kernel gave up waiting for its
// workgroups (d is then NaN).
constexpr int32_t kLanczosTimedOut = INT32_MIN;
struct LzLaunch {
    int cls, first, count, pmax;
};

// ------------------------------------------------------------------ handle
struct DevBuf {
    void *ptr = nullptr;
    size_t bytes = 0;
    int ensure(size_t need);   // grow (contents not kept); OEM_OK / OEM_E_NOMEM
    void release();
    template <typename T> T *as() const { return static_cast<T *>(ptr); }
};

// Device frees held back on one thread.  hipFree waits for the whole device,
// so a thread whose stream runs beside other streams (a worker of the request
// loop) would wait for their kernels each time it grows a buffer.  While a
// thread's deferred_frees is set, DevBuf::release hands its memory to the list
// instead; flush_deferred_frees frees it all (one wait for the device).
struct DeferredFrees {
    std::vector<void *> ptrs;
    size_t bytes = 0;
};
extern thread_local DeferredFrees *deferred_frees;
void flush_deferred_frees(DeferredFrees &d);

struct HostStage;   // staging of the out-of-core Gram pass (stream_host.hip)

// Small host tables a call uploads (groups, lambda values and penalties, path
// descriptors, the launch order).  Each slot keeps its bytes in the handle
// until the copy has run, so a call enqueues its uploads without waiting;
// the slot's event, recorded behind its copy, is waited for before the next
// call rewrites it.
enum UploadSlot { kUpGroups, kUpLambda, kUpDescs, kUpOrder, kUpSlots };
struct UploadStage {
    std::vector<char> bytes[kUpSlots];
    hipEvent_t done[kUpSlots] = {};
    bool pending[kUpSlots] = {};
};

} // namespace oem

struct oem_gram_s {
    int32_t p = 0, K = 1, prec = OEM_FP64, xdt = OEM_X_F32;
    uint64_t seed = 0;
    int device = 0;
    // raw per-fold sums
    oem::DevBuf Gk, bk, yyk, nk;       // K p^2, K p, K, K (int64)
    oem::DevBuf csk, ysk;              // column sums K p, sums of y K
    bool colsums_known = true;         // false once a fold was imported without them
    // derived problems: q = 0 full data, q = 1 + k training rows of fold k
    oem::DevBuf Gs, cs, sc, yyn, dq, ntrain, lzsteps;  // (K+1) p^2, (K+1) p, ...
    oem::DevBuf xbar, ybar;            // (K+1) p, K+1: means of the problem's rows (intercept)
    bool derived_valid = false;
    int derived_std = -1;
    int derived_icpt = -1;
    std::vector<double> d_host;        // d per problem (valid with derived_valid)
    std::vector<int64_t> n_host;       // rows per problem
    std::vector<int32_t> lz_host;      // Lanczos steps (negative: not converged)
    int64_t rows_seen = 0;
    // workspaces
    oem::DevBuf partial, partial_n, rowlist, lanczos, paths, order, lam, betaw, groupbuf, cvw, flag, pathws, lzjobs;
    oem::HostStage *stage = nullptr;   // out-of-core staging, created on first use
    oem::UploadStage up;               // host tables of the path calls
};

namespace oem {

// ------------------------------------------------------------------ launchers
int handle_reconfigure(oem_gram_s *h, int32_t p, int32_t K, int32_t prec, int32_t xdt, uint64_t seed,
                       hipStream_t s);
int launch_fill_f64(double *p, size_t n, double v, hipStream_t s);
int launch_fill_i64(int64_t *p, size_t n, int64_t v, hipStream_t s);
int launch_scale_f64(double *p, size_t n, double v, hipStream_t s);
// Device workspace of one Gram pass (row lists and partial sums).  With base
// set, the pass carves its buffers from [base, base + bytes) and allocates
// nothing; otherwise it grows the handle's own buffers.
struct GramWork {
    char *base = nullptr;
    size_t bytes = 0;
    size_t used = 0;
};
int launch_gram(oem_gram_s *g, const void *X, int64_t n, int64_t ldx, const double *y,
                int64_t row_offset, const uint8_t *foldid, hipStream_t s, GramWork *ws = nullptr);
int launch_gram_bf16(oem_gram_s *g, const void *X, int64_t n, int64_t ldx, const double *y,
                     int64_t row_offset, const uint8_t *foldid, hipStream_t s, GramWork *ws = nullptr);
// Weighted pass (FP64 form, one fold): the tiles accumulate sum_i w_i x_i x_i^T.
int launch_gram_weighted(oem_gram_s *h, const void *X, int64_t n, int64_t ldx, const double *y,
                         const double *wts, hipStream_t s);
// Penalised logistic paths (Section 4) on the rows X (n x ldx, the handle's
// element type), y in {0, 1}; the handle (p columns, one fold, FP64 form)
// is the workspace of the Gram passes and of d.
int logistic_path(oem_gram_s *h, const void *X, int64_t n, int64_t ldx, const double *y,
                  const oem_penalty *pen, int npen, const oem_path_opts *o, const oem_logistic_opts *lo,
                  const int32_t *d_gstart, const int32_t *d_gidx, int ngroups, const double *d_w,
                  const double *d_cg, double *beta, double *lambda, int32_t *newton_iters, double *kkt,
                  double *obj, hipStream_t s);
// Pass over sparse rows in compressed sparse row form (FP64 form only).
int launch_gram_csr(oem_gram_s *h, const int64_t *rowptr, const int32_t *col, const void *val, int64_t nnz,
                    int64_t n, const double *y, int64_t row_offset, const uint8_t *foldid, hipStream_t s);
// Out-of-core pass: rows of host-resident X (pageable, memory-mapped or
// pinned) streamed through pinned and device staging in chunks.
int gram_from_host(oem_gram_s *h, const void *X, int64_t n, int64_t ldx, const double *y,
                   int64_t row_offset, const uint8_t *foldid, int64_t chunk_rows, hipStream_t s);
void free_host_stage(oem_gram_s *h);
// Enqueue a copy of `bytes` host bytes to `dst` through upload slot `slot`
// of the handle (no host wait); release the slots' events.
int stage_upload(oem_gram_s *h, int slot, void *dst, const void *src, size_t bytes, hipStream_t s);
void free_upload_stage(oem_gram_s *h);
// Workspace bytes one Gram pass of the handle's shape over n rows carves
// from a GramWork (the same plan as the pass itself).
size_t gram_work_bytes(const oem_gram_s *h, int64_t n);
int launch_combine(oem_gram_s *g, int standardize, int intercept, hipStream_t s);
int launch_lanczos(oem_gram_s *g, hipStream_t s);
// Set on a thread whose Lanczos launches may run beside launches from other
// streams: every problem then uses one workgroup (no barrier across workgroups).
extern thread_local bool lanczos_single_workgroup;
int lanczos_mmax(int p);
size_t lanczos_workspace_doubles(int p);
// sort jobs by kernel class and cut them into launches
void lanczos_job_plan(std::vector<LzJob> &jobs, std::vector<LzLaunch> &launches);
int launch_lanczos_jobs(const LzJob *d_jobs, const std::vector<LzLaunch> &launches, hipStream_t s);
int launch_lambda_grid(const double *cs_full, int p, const int32_t *gstart, const int32_t *gidx,
                       int ngroups, const double *w, const double *cg, const oem_penalty *d_pens,
                       int npen, int L, double ratio, double *lambda_out, hipStream_t s);
int launch_paths(const PathDesc *d_desc, const std::vector<PathDesc> &host, DevBuf &orderbuf,
                 hipStream_t s, oem_gram_s *stage_owner);
// The same split into a plan (host: order table grouped by kernel class) and
// launches that enqueue kernels only (no allocation, no host wait).
// cls: path kernel; first: offset of its paths in the order table; chain:
// the kernel continues the paths of an earlier launch from their hand-over
struct PathLaunch {
    int cls, first, count, pmax, chain;
};
struct PathPlan {
    std::vector<int> order;
    std::vector<PathLaunch> launches;
};
void plan_paths(const std::vector<PathDesc> &host, PathPlan &plan);
// hand-over buffers of the paths: lstart and bws of every descriptor point into buf
int attach_path_handover(std::vector<PathDesc> &descs, DevBuf &buf);
int launch_paths_planned(const PathDesc *d_desc, const int *d_order, const PathPlan &plan,
                         hipStream_t s);
int launch_cv(const double *Gk, const double *bk, const double *yyk, const int64_t *nk,
              const double *csk, const double *ysk, const double *beta0_folds,
              int K, int p, int npen, int L, const double *beta_folds, double *mse,
              double *cvm, double *cvsd, int32_t *i_min, int32_t *i_1se, int32_t *best,
              hipStream_t s);
// One path of the general kernel per descriptor d_desc[0 .. count) (no
// order table), e.g. single-lambda solves from a warm start.
int launch_paths_general(const PathDesc *d_desc, int count, int pmax, hipStream_t s);
// intercepts ybar - xbar^T beta of every path whose descriptor asks for them
int launch_intercepts(const PathDesc *d_desc, int count, hipStream_t s);

} // namespace oem
