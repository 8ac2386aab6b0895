/*
 * oem.h - C ABI of the MI355X (gfx950) OEM library for penalized least
 * squares on tall data.
 *
 * Method: orthogonalizing EM (OEM) as reviewed in Huling & Qian, "Fast
 * Penalized Regression and Cross Validation for Tall Data with the oem
 * Package", Section 2.  The problem (Section 2.1, eq. (eqn:pen_loss), with
 * the 1/n scaling of the precomputed-statistics interface of Section 5.6) is
 *
 *     minimise_beta  1/(2n) ||y - X beta||^2 + P_lambda(beta)
 *
 * for X n x p (n >> p).  Everything the iteration needs is in the sufficient
 * statistics G = X^T X, X^T y, y^T y and n; for K-fold cross validation the
 * per-fold statistics are summed to give each training Gram (Section 3).
 *
 * Library flow:
 *   oem_gram_create      one handle per (p, K, precision)
 *   oem_gram             one streaming pass over a block of rows (may be
 *                        repeated on successive row blocks; sums accumulate)
 *   oem_fit_path         warm-started lambda path(s) on all rows or on the
 *                        training rows of one fold
 *   oem_cv               paths on every fold plus the full data, held-out
 *                        error and model selection
 *   oem_gram_free
 *
 * Conventions shared by every entry point
 *   - Return value: OEM_OK (0), OEM_NOT_CONVERGED (1, a warning: outputs are
 *     valid) or a negative error code; oem_last_error() gives a message for
 *     the calling thread's last non-OK return.
 *   - "device pointer": memory the GPU can read or write (hipMalloc'd, or
 *     pinned host memory from hipHostMalloc).  "host pointer": ordinary CPU
 *     memory, read during the call only.
 *   - The caller owns every pointer it passes; the library never keeps one
 *     after the call returns.  The handle owns its own device buffers.
 *   - stream: a hipStream_t passed as void* (NULL = the null stream).  Work
 *     is enqueued on it; device outputs are valid after the stream is
 *     synchronised.  A handle must not be used from two threads at once.
 *   - Host waits.  oem_gram, oem_gram_reset, oem_gram_import,
 *     oem_gram_export and oem_batch_run(_graph) enqueue work and return
 *     without waiting for the GPU.  oem_fit_path and oem_cv wait for
 *     `stream` once after the statistics changed, to read back d and the
 *     row counts they validate (penalty conditions gamma d > 1, empty
 *     folds).  Their small host tables (lambda values, groups, path
 *     descriptors, a few KB) are copied into the handle and uploaded
 *     without a wait (a later call waits, if need be, for the previous
 *     upload of the same table before reusing its host copy); the path, CV
 *     and selection kernels are enqueued and the call returns before they
 *     finish unless opts->sync = 1.  oem_gram_autotune,
 *     oem_batch_create, oem_batch_status and the free functions wait for
 *     the device.
 *   - Concurrent streams.  For 128 < p <= 2048 the eigenvalue bound d is
 *     computed by launches whose workgroups exchange data every step, so all
 *     workgroups of a launch must be resident at once; each launch of
 *     oem_fit_path / oem_cv takes at most half of the CUs (by the occupancy
 *     of an idle device; a batch's launches take all of them, so a batch
 *     run has the GPU to itself while it derives d).  Other work
 *     that runs at the same time and finishes by itself (a Gram pass or the
 *     paths of another handle on another stream) can delay such a launch
 *     but not stop it, and two such launches fit side by side.  More than
 *     two at once (three or more handles deriving d on concurrent streams)
 *     can keep each other's workgroups waiting: the bounded waits then end
 *     and oem_fit_path / oem_cv return OEM_E_HIP ("timed out waiting for its
 *     workgroups"), never a hang or a wrong d.  Such callers set the
 *     environment variable OEM_LANCZOS_MB=0 before the first call (one
 *     workgroup per problem, no cross-workgroup wait); the request loop's
 *     workers (oem_server_*) always use one workgroup per problem.
 *   - Matrices are row-major.  Sizes are element counts.
 */
#ifndef OEM_H
#define OEM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes. */
enum {
    OEM_OK = 0,
    OEM_NOT_CONVERGED = 1, /* some (path, lambda) hit maxit; iters < 0 there */
    OEM_E_INVAL = -1,      /* invalid argument */
    OEM_E_NOMEM = -2,      /* device allocation failed */
    OEM_E_HIP = -3,        /* a HIP runtime call failed */
    OEM_E_STATE = -4       /* handle not in a state that allows the call */
};

/* Arithmetic of the Gram pass and of the path iterations.
 *   OEM_FP64        X widened to FP64, FP64 matrix-core products, FP64 paths.
 *   OEM_SPLIT_BF16  x = hi + lo (two BF16 parts), three BF16 products
 *                   (hi*hi + hi*lo + lo*hi) accumulated in FP32 on the matrix
 *                   cores, flushed to FP64 and summed over row splits in
 *                   FP64; the diagonal, X^T y and y^T y in FP64.  Everything
 *                   after the Gram pass (standardisation, d, the paths, CV)
 *                   is FP64, exactly as in OEM_FP64, on this Gram.  A pass
 *                   (one oem_gram call, one out-of-core chunk) over fewer
 *                   than 32768 rows forms its products in FP64 instead: the
 *                   BF16 rounding errors average over too few rows there to
 *                   keep coefficients within 1e-6 of the FP64 form.
 *   OEM_BF16        as SPLIT_BF16 with the hi part only (reported variant). */
enum { OEM_FP64 = 0, OEM_SPLIT_BF16 = 1, OEM_BF16 = 2 };

/* Element type of X. */
enum { OEM_X_F32 = 0, OEM_X_F64 = 1 };

/* Penalties (Section 2.2, penalty table; updates eqs. lasso, net, mcp, scad,
 * glasso, gmcp, gscad, sglasso).  Group penalties need a group partition.
 * Group MCP / SCAD are sum_k P_{lambda c_k, gamma}(||beta_{g_k}||) (the
 * table's extra factor lambda read as a typo): the update scales u_g by the
 * scalar MCP / SCAD update of ||u_g|| at c_k lambda.  The sparse group lasso
 * update soft-thresholds each u_j at w_j lambda tau and applies the group
 * lasso update at c_k lambda (1 - tau), both with the same d: the proximal
 * map of the nested penalty (the printed form differs unless d = 1). */
enum {
    OEM_LASSO = 0,     /* lambda sum_j w_j |beta_j|                         */
    OEM_ENET = 1,      /* alpha lambda sum w|b| + (1-alpha)/2 lambda sum w b^2 */
    OEM_MCP = 2,       /* minimax concave penalty, gamma > 1                */
    OEM_SCAD = 3,      /* smoothly clipped absolute deviation, gamma > 2    */
    OEM_GRP_LASSO = 4, /* lambda sum_k c_k ||beta_{g_k}||                   */
    OEM_GRP_MCP = 5,   /* sum_k P^MCP_{lambda c_k, gamma}(||beta_{g_k}||), gamma > 1 */
    OEM_GRP_SCAD = 6,  /* sum_k P^SCAD_{lambda c_k, gamma}(||beta_{g_k}||), gamma > 2 */
    OEM_SGL = 7        /* lambda (1-tau) sum_k c_k ||beta_g|| + lambda tau sum_j w_j |beta_j| */
};

typedef struct {
    int32_t kind;  /* OEM_LASSO .. OEM_SGL */
    double alpha;  /* elastic net mixing, 0 < alpha <= 1 (ignored otherwise) */
    double gamma;  /* (group) MCP / SCAD concavity (ignored otherwise) */
    double tau;    /* sparse group lasso mixing, 0 <= tau <= 1; must be 0 for
                      every other kind */
} oem_penalty;

/* Options of a path fit.  Every pointer here is a HOST pointer, except beta0
 * (a device output). */
typedef struct {
    int32_t nlambda;          /* L >= 1 values per penalty                        */
    double lambda_min_ratio;  /* lambda_L / lambda_1 in (0, 1] when lambda == NULL */
    const double *lambda;     /* npen x L explicit sequences, or NULL: log grid
                                 from lambda_max of the full-data statistics      */
    double tol;               /* stop when max|delta beta| <= tol * max|beta|     */
    int32_t maxit;            /* OEM updates per lambda, >= 1                     */
    int32_t standardize;      /* 1: columns scaled to unit norm (Section 2.1)     */
    const int32_t *groups;    /* p group ids in [0, ngroups), every id used; NULL
                                 allowed unless a group penalty is requested      */
    const double *w;          /* p variable weights >= 0, NULL = all 1            */
    const double *cg;         /* ngroups group weights > 0, NULL = sqrt(size)     */
    int32_t sync;             /* 1: wait for the stream and return
                                 OEM_NOT_CONVERGED when some lambda hit maxit     */
    int32_t intercept;        /* 1: unpenalised intercept.  The columns and y are
                                 centred with the means of the rows fitted (the
                                 training rows of a fold), from the column sums
                                 the Gram pass accumulates: G/n - xbar xbar^T,
                                 X^T y/n - xbar ybar, y^T y/n - ybar^2 (no
                                 intercept in the model of Section 2.1; this is
                                 the glmnet-style option).  Standardisation then
                                 uses the centred column norms.  Cancellation:
                                 relative accuracy of the centred Gram is about
                                 1e-16 (xbar^2 / variance).  Not available after
                                 oem_gram_import (no column sums).  0: none.     */
    double *beta0;            /* DEVICE output npen x L: intercepts
                                 ybar - xbar^T beta (original scale) of the
                                 full-data or fold paths fitted; NULL allowed    */
} oem_path_opts;

typedef struct oem_gram_s *oem_handle;

/* Create a handle for p columns and nfolds folds (1 = no cross validation).
 * precision: OEM_FP64 | OEM_SPLIT_BF16 | OEM_BF16.  x_dtype: OEM_X_F32 |
 * OEM_X_F64.  fold_seed: seed of the fold hash (Section 3 partitions the rows
 * at random): row i (global index) is in fold floor(nfolds * h_i / 2^32),
 * h_i = high 32 bits of the (i+1)-th SplitMix64 output from state fold_seed.
 * Uses the current HIP device.  Errors: OEM_E_INVAL (p < 1, p > 4096,
 * nfolds < 1 or > 64, bad enum), OEM_E_NOMEM, OEM_E_HIP. */
int oem_gram_create(int32_t p, int32_t nfolds, int32_t precision, int32_t x_dtype,
                    uint64_t fold_seed, oem_handle *out);

/* Release the handle and its device memory (NULL is ignored).  Waits for
 * work already enqueued with the handle. */
void oem_gram_free(oem_handle g);

/* Set every accumulated statistic back to zero. */
int oem_gram_reset(oem_handle g, void *stream);

/* One streaming pass over rows 0..n-1 of X (device pointer, n x p, row
 * stride ldx >= p elements of the handle's x_dtype) and y (device pointer,
 * n FP64 values), adding to the per-fold sums (Section 3):
 *     G_k += sum_{i in fold k} x_i x_i^T,  b_k += sum x_i y_i,
 *     yy_k += sum y_i^2,                   n_k += |{i in fold k}|.
 * row_offset: global index of row 0 (the fold hash uses global indices, so
 * successive blocks of one data set keep their folds).  foldid: NULL (use
 * the hash) or a device array of n fold ids; rows whose id is >= nfolds are
 * skipped.  n = 0 is a no-op; one call takes at most 2^31 - 1 rows (pass
 * larger data sets as successive blocks).  X and y are not referenced after
 * the work completes.  The BF16 forms take FP32 X only.  Errors: OEM_E_INVAL
 * (NULL X or y with n > 0, ldx < p, n < 0 or too large, FP64 X with a BF16
 * form), OEM_E_HIP. */
int oem_gram(oem_handle g, const void *X, int64_t n, int64_t ldx, const double *y,
             int64_t row_offset, const uint8_t *foldid, void *stream);

/* One streaming pass over sparse rows (Section 5.8: sparse design
 * matrices) in compressed sparse row form, FP64 Gram form only.  Row i
 * (0 <= i < n) stores the entries t in [rowptr[i], rowptr[i + 1]) at
 * columns colidx[t] with values values[t] (element type of the handle's
 * x_dtype); columns outside [0, p) are ignored, repeated columns add.  Device
 * pointers: rowptr (n + 1 int64), colidx and values (nnz), y (n), foldid
 * (n, or NULL).  Each row block is densified in LDS and goes through the
 * same matrix-core tiles as oem_gram, so the sums equal oem_gram's on the
 * densified rows bit for bit; only the stored entries are read from memory.
 * Entry ranges are clamped to [0, nnz), so a malformed rowptr gives
 * meaningless sums but no out-of-range reads.  Accumulates like oem_gram.
 * Errors: OEM_E_INVAL (NULL pointers, n or nnz negative, n > 2^31 - 1, a
 * BF16 form), OEM_E_HIP. */
int oem_gram_csr(oem_handle g, const int64_t *rowptr, const int32_t *colidx, const void *values,
                 int64_t nnz, int64_t n, const double *y, int64_t row_offset, const uint8_t *foldid,
                 void *stream);

/* Out-of-core pass (Section 5.7: data larger than memory, e.g. a memory-
 * mapped file): the rows 0..n-1 of host-resident X (HOST pointer: ordinary,
 * memory-mapped or pinned memory; n x p, row stride ldx >= p) and y (host,
 * n FP64), with optional host fold ids, stream through two pinned staging
 * slots and two device slots of chunk_rows rows each.  Packing a chunk on
 * the CPU (skipped when X is pinned), its host-to-device copy on a copy
 * stream of the handle and the Gram kernels of the previous chunk on
 * `stream` overlap.  Each chunk is one accumulating pass with its global row
 * offset (row_offset + its first row), so the sums are those of oem_gram
 * called on the same blocks, and n may exceed 2^31 - 1.  Device memory: two
 * chunks (chunk_rows (p sizeof(x) + 9) bytes each) plus the pass workspace,
 * not n p.  Returns once every chunk has been copied (the host arrays are
 * not read afterwards); the Gram kernels may still run on `stream`.  The
 * first call (or a new chunk size) allocates the staging: pinned host and
 * device memory, kept with the handle until oem_gram_free.
 * Errors: as oem_gram; OEM_E_INVAL also when X, y or foldid is device memory
 * or chunk_rows is not in [1, 2^31 - 1]; OEM_E_NOMEM. */
int oem_gram_host(oem_handle g, const void *X, int64_t n, int64_t ldx, const double *y,
                  int64_t row_offset, const uint8_t *foldid, int64_t chunk_rows, void *stream);

/* oem_gram for callers that cannot allocate device memory: code under
 * hipGraph capture, request loops that must not call hipMalloc, harnesses
 * that forbid it.  Same arguments, sums and kernels as oem_gram; the pass's
 * row lists and partial sums live in a static device workspace of 64 MiB
 * (one per device, held until the process ends) instead of buffers the
 * handle grows, so the call allocates nothing (the handle's sums were
 * allocated by oem_gram_create).  Every call on one device shares that
 * device's workspace: calls that overlap in time on one device (two host
 * threads, or two streams whose work runs concurrently) race and must be
 * serialised by the caller.  The workspace needs no clearing between calls.
 * Errors: as oem_gram; OEM_E_INVAL when the current device is not the
 * handle's, or when the pass needs more than the workspace (with folds the
 * row lists take 4 bytes per row: pass larger data sets as successive row
 * blocks). */
int oem_gram_noalloc(oem_handle g, const void *X, int64_t n, int64_t ldx, const double *y,
                     int64_t row_offset, const uint8_t *foldid, void *stream);

/* Load sufficient statistics computed elsewhere into fold slot `fold`
 * (precomputed X^T X and X^T y, Section 5.6).  XtX (p x p), Xty (p): device
 * pointers.  scaled = 1: the inputs are X^T X / n, X^T y / n, y^T y / n (the
 * scaling used in Section 5.6) and are multiplied by n; scaled = 0: raw sums.
 * Replaces the slot's previous contents.  Errors: OEM_E_INVAL. */
int oem_gram_import(oem_handle g, int32_t fold, const double *XtX, const double *Xty,
                    double yty, int64_t n, int32_t scaled, void *stream);

/* Copy the raw per-fold sums out: G (nfolds x p x p), b (nfolds x p), yy
 * (nfolds), nk (nfolds).  Device pointers; any may be NULL. */
int oem_gram_export(oem_handle g, double *G, double *b, double *yy, int64_t *nk, void *stream);

/* Copy the per-fold column sums sum_{i in k} x_i (nfolds x p) and sums of y
 * (nfolds) out (device pointers, either may be NULL); the intercept option
 * centres with them.  Errors: OEM_E_STATE after oem_gram_import (imported
 * statistics carry no column sums). */
int oem_gram_export_colsums(oem_handle g, double *colsum, double *ysum, void *stream);

/* Warm-started OEM paths (Section 2.1 iteration, Section 2.2 updates) for
 * npen penalties (host array) on the full data (fold = -1) or on the rows
 * outside fold `fold` (its training rows, Section 3).
 * Per penalty: beta = 0, then for each lambda in order repeat
 *     u = c + (d I - G) beta,   beta <- update_penalty(u, lambda, d)
 * until max_j |delta beta_j| <= tol * max_j |beta_j| or maxit updates, with G,
 * c the (standardised) Gram and X^T y scaled by 1/n and d = lambda_1(G) *
 * (1 + 1e-10) from a Lanczos eigen-solve.
 * Device outputs (any may be NULL except beta):
 *     beta    npen x L x p   coefficients on the original scale of X
 *     lambda  npen x L       the lambda sequence used
 *     iters   npen x L       updates used; -maxit where maxit was reached
 *     kkt     npen x L       max stationarity violation (standardised scale)
 *     obj     npen x L       objective value
 *     d_out   1              the d used
 * d: when the Lanczos iteration does not settle within its step limit, d is
 * the Gershgorin bound max_i sum_j |G_ij| instead (still >= lambda_1).
 * Errors: OEM_E_INVAL (fold out of range, n of the selected rows = 0, bad
 * penalty parameters: alpha not in (0,1], (group) MCP gamma <= 1 or
 * gamma d <= 1, (group) SCAD gamma <= 2 or (gamma-1) d <= 1, tau not in
 * [0, 1] or nonzero outside the sparse group lasso, bad groups, L < 1,
 * maxit < 1; d not
 * a finite positive number, i.e. non-finite or all-zero statistics),
 * OEM_E_STATE (no rows accumulated), OEM_E_HIP (including an eigenvalue
 * solve whose workgroups could not all run at once). */
int oem_fit_path(oem_handle g, int32_t fold, const oem_penalty *pen, int32_t npen,
                 const oem_path_opts *opts, double *beta, double *lambda, int32_t *iters,
                 double *kkt, double *obj, double *d_out, void *stream);

/* K-fold cross validation from the fold statistics (Section 3; outputs as in
 * Section 5.5): paths on the full data and on each fold's training rows with
 * the full-data lambda sequence, held-out mean squared error of each fold
 *     MSE_{k,l} = (yy_k - 2 beta_l^T b_k + beta_l^T G_k beta_l) / n_k,
 * cvm_l = sum_k n_k MSE_{k,l} / n,
 * cvsd_l = sqrt(sum_k n_k (MSE_{k,l} - cvm_l)^2 / (n (K - 1))),
 * i_min = first argmin of cvm, i_1se = first l with cvm_l <= cvm_min + cvsd at
 * i_min, best = penalty with the smallest minimum cvm (first on ties).
 * Device outputs (NULL allowed except beta_full, cvm):
 *     beta_full  npen x L x p        full-data coefficients
 *     beta_folds K x npen x L x p    training-row coefficients of each fold
 *     lambda     npen x L
 *     cvm, cvsd  npen x L
 *     i_min, i_1se npen;  best 1
 *     iters      (K + 1) x npen x L  (slot 0 = full data)
 * Requires nfolds >= 2.  Errors as oem_fit_path, and OEM_E_INVAL when a fold
 * has no held-out rows (n_k = 0, e.g. a fold-id array that skips an id). */
int oem_cv(oem_handle g, const oem_penalty *pen, int32_t npen, const oem_path_opts *opts,
           double *beta_full, double *beta_folds, double *lambda, double *cvm, double *cvsd,
           int32_t *i_min, int32_t *i_1se, int32_t *best, int32_t *iters, void *stream);

/* Time the Gram pass of this handle's shape on the rows (X, n, ldx, y) (as
 * oem_gram: device pointers, row-major) for several workgroup counts, keep
 * the fastest for every later pass of the same (precision, folds, p rounded
 * up to 32, floor(log2 n)) shape in this process, then clear the handle's
 * sums as oem_gram_reset does.  Waits for `stream`.
 * Errors: as oem_gram. */
int oem_gram_autotune(oem_handle g, const void *X, int64_t n, int64_t ldx, const double *y,
                      void *stream);

/* ------------------------------------------------------------------ logistic
 * Penalised logistic regression (Section 4).  y_i in {0, 1}, Pr(y_i = 1) =
 * 1 / (1 + exp(-x_i^T beta)), no intercept; minimise the mean negative
 * log-likelihood (1/n) sum [log(1 + exp(x_i^T beta)) - y_i x_i^T beta] plus
 * the penalty (the printed log-likelihood's signs read as the standard
 * ones).  Proximal Newton (Friedman, Hastie & Tibshirani 2010) with OEM as
 * the inner solver: at the current beta the working weights mu (1 - mu)
 * (hessian_bound = 1: the bound 1/4 for every row, which keeps one Gram for
 * the whole path and turns the steps into a majorise-minimise iteration)
 * give the weighted least-squares model, minimised by OEM updates (opts tol
 * and maxit) from the current point with d = lambda_1 (1 + 1e-10) of its
 * standardised Hessian; Newton steps repeat until max|delta beta| <=
 * newton_tol max|beta|.  Columns are standardised once to unit mean square
 * (opts->standardize must be 1).  Warm starts along lambda; one grid per
 * penalty from lambda_max of X~^T (y - 1/2) / n unless opts->lambda is set. */
typedef struct {
    int32_t hessian_bound;  /* 1: w_i = 1/4; 0: exact weights mu (1 - mu)   */
    double newton_tol;      /* > 0                                          */
    int32_t newton_maxit;   /* >= 1                                         */
} oem_logistic_opts;

/* Logistic paths for npen penalties on X (device, n x p, row stride ldx,
 * element type x_dtype) and y (device, n values in {0, 1}).  Device outputs
 * (NULL allowed except beta): beta npen x L x p (original scale), lambda
 * npen x L, newton_iters npen x L (Newton steps; negative at newton_maxit),
 * kkt npen x L (stationarity violation of the logistic problem), obj npen x
 * L.  Waits for `stream` after every Newton step (the stopping test) and
 * before returning.  Allocates its workspace (a handle's buffers and n + 512
 * p doubles) for the call.  p <= 2048.  Not covered: intercept, CV (the
 * fold-Gram shortcut of Section 3 does not apply), the BF16 forms.
 * Errors: OEM_E_INVAL (shapes, options, penalties as oem_fit_path, MCP /
 * SCAD conditions checked against d at every step), OEM_E_NOMEM, OEM_E_HIP;
 * OEM_NOT_CONVERGED when some lambda hit newton_maxit (outputs valid). */
int oem_logistic_path(const void *X, int32_t x_dtype, int64_t n, int64_t ldx, int32_t p, const double *y,
                      const oem_penalty *pen, int32_t npen, const oem_path_opts *opts,
                      const oem_logistic_opts *lopts, double *beta, double *lambda, int32_t *newton_iters,
                      double *kkt, double *obj, void *stream);

/* ------------------------------------------------------------------ batches
 * Many independent tall problems of uneven p fitted together (the same
 * penalties and path options for all).  Each problem is either the
 * full-data fit of oem_fit_path (Gram pass, standardisation, d, lambda grid,
 * warm-started paths) or, with nfolds >= 2, the K-fold cross validation of
 * oem_cv from per-fold Grams (Section 3: the fold sums of one pass give every
 * training Gram; folds x penalties x lambda paths, held-out error and the
 * selection).  All problems' d (every fold's too) are found by one Lanczos
 * launch per kernel class and all (problem, fold, penalty) paths by one path
 * launch per kernel class, so the launch count does not grow with the number
 * of problems or folds. */
typedef struct {
    int32_t p;            /* columns, 1..4096 */
    int64_t n;            /* rows, 1..2^31-1 */
    int64_t ldx;          /* row stride of X, >= p */
    const void *X;        /* device, n x ldx row-major, element type x_dtype */
    const double *y;      /* device, n */
    double *beta;         /* device output, npen x L x p (original scale; the
                             full-data paths) */
    double *lambda;       /* device output, npen x L, or NULL */
    int32_t *iters;       /* device output, npen x L (nfolds <= 1) or
                             (K + 1) x npen x L (full data first, as oem_cv),
                             or NULL */
    double *kkt;          /* device output, npen x L (full data), or NULL */
    double *obj;          /* device output, npen x L (full data), or NULL */
    /* cross validation, groups and explicit lambda (zero / NULL: none) */
    int32_t nfolds;       /* 0 or 1: full-data fit; 2..64: K-fold CV */
    uint64_t fold_seed;   /* fold hash seed (nfolds >= 2) */
    const int32_t *groups;    /* host, p group ids in [0, ngroups), every id
                                 used (needed by group penalties), or NULL;
                                 read by oem_batch_create only */
    const double *lambda_in;  /* host, npen x L lambda values >= 0 used
                                 instead of the grid, or NULL; read by
                                 oem_batch_create only */
    double *beta_folds;   /* device output, K x npen x L x p (training rows
                             of fold k), or NULL */
    double *cvm;          /* device output, npen x L: CV error (required when
                             nfolds >= 2) */
    double *cvsd;         /* device output, npen x L, or NULL */
    int32_t *i_min;       /* device output, npen, or NULL */
    int32_t *i_1se;       /* device output, npen, or NULL */
    int32_t *best;        /* device output, 1 value (penalty of the smallest
                             cvm), or NULL */
} oem_problem;

typedef struct oem_batch_s *oem_batch;

/* Plan a batch: copies the nprob problem records (their X, y and output
 * pointers must stay valid while the batch is used; groups and lambda_in are
 * read here only), creates every device buffer, tunes the Gram pass of each
 * problem shape with n p >= 2^22 (oem_gram_autotune), and runs the batch
 * once on the null stream, after which every cross-validation problem's
 * folds are checked for training and held-out rows.
 * Restrictions: opts->standardize = 1 (then d >= 1, so the MCP and SCAD
 * conditions on gamma d hold for every problem), no intercept, and the
 * per-problem fields instead of opts->groups, opts->lambda, opts->w and
 * opts->cg (which must be NULL; group weights are sqrt(group size)).  Group
 * penalties need every problem's groups.
 * Errors: OEM_E_INVAL (bad problem record or option, nprob < 1, a fold with
 * no training or no held-out rows), OEM_E_NOMEM, OEM_E_HIP. */
int oem_batch_create(const oem_problem *probs, int32_t nprob, int32_t precision, int32_t x_dtype,
                     const oem_penalty *pen, int32_t npen, const oem_path_opts *opts,
                     oem_batch *out);

/* Enqueue the whole batch on `stream`: per problem a Gram pass from zero
 * sums (with fold sums for CV problems) and the standardisation of every
 * fold, then the batched Lanczos, lambda-grid and path launches, then per CV
 * problem the held-out error and selection kernels.  Kernels and
 * device-to-device copies only: no allocation and no host wait, so the
 * sequence may be captured into a hipGraph. */
int oem_batch_run(oem_batch b, void *stream);

/* The work of oem_batch_run captured into a hipGraph on the first call (on
 * `stream`) and replayed with hipGraphLaunch on every call. */
int oem_batch_run_graph(oem_batch b, void *stream);

/* Wait for `stream`; OEM_NOT_CONVERGED if some lambda of some problem reached
 * maxit in the last run, else OEM_OK. */
int oem_batch_status(oem_batch b, void *stream);

/* Release the batch's device buffers and graph (waits for the device). */
void oem_batch_free(oem_batch b);

/* ------------------------------------------------------------------ serving
 * A request loop that keeps a number of fit and cross-validation requests
 * of differing n and p in flight at once.  Each of `nslots` worker threads
 * owns a stream and its device buffers; a request is admitted when a slot is
 * free and the device bytes of the requests in flight plus its own stay
 * within `device_bytes` (a request larger than the budget runs alone), in
 * arrival order.  A request is: copy of X, y to the device (when they are
 * host memory), Gram pass (with fold statistics for CV), and the full-data
 * path of oem_fit_path or the cross validation of oem_cv, outputs copied to
 * the caller's host arrays.  Requests in flight overlap on the device; each
 * result is the one the request gives alone (same kernels, same inputs).
 * Device memory: a worker keeps its buffers between requests.  Its staging
 * of X, y and the outputs is released after a request when it passes the
 * worker's share of the budget (device_bytes / nslots); its Gram statistics
 * and path workspace, which grow with p^2 and the folds but not with n, keep
 * the size of the largest request it has seen.  hipFree waits for the whole
 * device, so the buffers a request outgrows are freed between requests, once
 * they pass a quarter of that share, and during a request only when an
 * allocation fails without them. */
typedef struct {
    int64_t id;                /* caller's tag, returned in the completion */
    int32_t p;                 /* columns, 1..4096 */
    int64_t n;                 /* rows, 1..2^31-1 */
    int64_t ldx;               /* row stride of X, >= p */
    const float *X;            /* FP32 rows: host (pinned: asynchronous copy) or device */
    const double *y;           /* n responses: host or device */
    int32_t nfolds;            /* 1: fit on all rows; 2..64: K-fold cross validation */
    uint64_t fold_seed;        /* fold hash seed (cross validation) */
    oem_penalty pen;           /* one penalty */
    const int32_t *groups;     /* host, p group ids (group lasso), else NULL */
    double *beta;              /* host output, L x p: full-data path, original scale */
    double *lambda;            /* host output, L, or NULL */
    double *cvm;               /* host output, L (cross validation), or NULL */
    int32_t *i_min;            /* host output, 1 (cross validation), or NULL */
    double t_arrival;          /* arrival time on the oem_server_now clock; < 0: submit time */
} oem_request;

typedef struct {
    int64_t id;
    int32_t status;            /* OEM_OK, OEM_NOT_CONVERGED or a negative error code */
    int32_t slot;              /* worker that ran it */
    double t_arrival, t_admit, t_done;   /* seconds on the oem_server_now clock */
    int64_t bytes;             /* device bytes it was admitted with */
} oem_completion;

typedef struct oem_server_s *oem_server;

/* Start the workers.  opts: the path options of every request (lambda,
 * groups, w, cg must be NULL; a request's groups come with the request).
 * Errors: OEM_E_INVAL (nslots not in 1..16, device_bytes < 1, bad opts). */
int oem_server_create(int32_t nslots, int64_t device_bytes, int32_t precision,
                      const oem_path_opts *opts, oem_server *out);

/* Queue a request (copied; its host arrays must stay valid until its
 * completion is returned).  Thread-safe.  Errors: OEM_E_INVAL (bad shape,
 * pointer or fold count). */
int oem_server_submit(oem_server s, const oem_request *req);

/* Move up to `max` completions into out (host array), their number into
 * *count; with wait != 0, block until at least one is available or nothing
 * is queued or running. */
int oem_server_poll(oem_server s, oem_completion *out, int32_t max, int32_t *count, int32_t wait);

/* Block until every submitted request has completed. */
int oem_server_drain(oem_server s);

/* Seconds on the server's monotonic clock. */
double oem_server_now(void);

/* Stop the workers after the queued requests and release everything. */
void oem_server_free(oem_server s);

/* Message for the calling thread's last non-OK return ("" if none). */
const char *oem_last_error(void);

/* Library version string. */
const char *oem_version(void);

#ifdef __cplusplus
}
#endif
#endif /* OEM_H */
