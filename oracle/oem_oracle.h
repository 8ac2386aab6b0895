/*
 * OEM oracle: plain, slow, FP64 CPU reference for the OEM penalized
 * least-squares path (Huling & Qian, "Fast Penalized Regression and Cross
 * Validation for Tall Data with the oem Package").
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this code; only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg use it.  It shares no source, header, table or helper with
 * the GPU library.
 *
 * Every routine is a direct transcription of the definition it cites:
 * naive loops in double precision, no blocking, no fusion, no reordering.
 *
 * Problem statement (Section 2.1, eq. (eqn:pen_loss) and the M-step (mstep)),
 * with the 1/n scaling of the precomputed-statistics interface (Section 5.6):
 *     minimise  1/(2n) ||y - X beta||^2 + P_lambda(beta)
 * which in Gram form, with G = X^T X / n and c = X^T y / n, is
 *     f(beta) = 1/2 beta^T G beta - c^T beta + 1/2 y^T y / n + P_lambda(beta).
 */
#ifndef OEM_ORACLE_H
#define OEM_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORACLE_LASSO = 0, ORACLE_ENET = 1, ORACLE_MCP = 2, ORACLE_SCAD = 3, ORACLE_GRP_LASSO = 4,
       ORACLE_GRP_MCP = 5, ORACLE_GRP_SCAD = 6, ORACLE_SGL = 7 };

typedef struct {
    int32_t kind;   /* ORACLE_* */
    double alpha;   /* elastic net mixing, 0 < alpha <= 1 */
    double gamma;   /* MCP / group MCP (> 1) or SCAD / group SCAD (> 2) concavity */
    double tau;     /* sparse group lasso mixing, 0 <= tau <= 1 */
} oracle_penalty;

/* ---- fold assignment (Section 3: rows randomly partitioned into K folds) ----
 * SplitMix64 (Steele, Lea & Flood 2014): state += 0x9E3779B97F4A7C15, output
 * = mix64(state).  Row i (global index) is the (i+1)-th output from state =
 * seed; its fold is the high 32 bits scaled to [0, K) by a 32x32 multiply. */
uint64_t oracle_splitmix64_next(uint64_t *state);
int32_t oracle_fold_of_row(uint64_t seed, int64_t i, int32_t K);
/* Folds of rows row_offset .. row_offset + n - 1 into out (n bytes). */
void oracle_fold_ids(uint64_t seed, int64_t row_offset, int64_t n, int32_t K, uint8_t *out);

/* ---- sufficient statistics (Section 3) ----
 * Per fold k: G_k = sum_{i in k} x_i x_i^T (p x p), b_k = sum x_i y_i,
 * yy_k = sum y_i^2, n_k = |fold k|.  Un-normalised sums.  X is row-major with
 * row stride ldx, FP32 (x_is_f64 = 0, widened exactly) or FP64.  Row i's fold
 * is foldid[i] when foldid != NULL, else the hash of (fold_seed,
 * row_offset + i); K = 1 puts every row in fold 0. */
int oracle_gram_folds(const void *X, int32_t x_is_f64, int64_t n, int64_t ldx, int32_t p,
                      const double *y, int64_t row_offset, int32_t K, uint64_t fold_seed,
                      const uint8_t *foldid, double *G, double *b, double *yy, int64_t *nk);

/* The same per-fold sums from sparse rows (Section 5.8) in compressed sparse
 * row form: row i stores val[t] at column col[t] for t in [rowptr[i],
 * rowptr[i + 1]); the products of every pair of stored entries of a row are
 * added (repeated columns add).  Returns -1 for a column outside [0, p) or
 * a decreasing rowptr. */
int oracle_gram_csr(const int64_t *rowptr, const int32_t *col, const double *val, int64_t n, int32_t p,
                    const double *y, int64_t row_offset, int32_t K, uint64_t fold_seed,
                    const uint8_t *foldid, double *G, double *b, double *yy, int64_t *nk);

/* Gram of the training rows of fold k directly (rows whose fold != k;
 * k = -1: every row).  One p x p output. */
int oracle_gram_train(const void *X, int32_t x_is_f64, int64_t n, int64_t ldx, int32_t p,
                      const double *y, int64_t row_offset, int32_t K, uint64_t fold_seed,
                      const uint8_t *foldid, int32_t k, double *G, double *b, double *yy,
                      int64_t *ntrain);

/* ---- standardisation (Section 2.1: unit column norms) ----
 * s_j = sqrt(G_jj) (1 if G_jj <= 0); Gs = S^-1 G S^-1, cs = S^-1 c. */
void oracle_standardize(int32_t p, const double *G, const double *c, double *Gs, double *cs,
                        double *s);

/* ---- d >= largest eigenvalue (Section 2.1, active orthogonalisation) ----
 * All eigenvalues of a symmetric matrix by the cyclic Jacobi method.
 * Returns the number of sweeps, or -1 if it did not converge. */
int oracle_sym_eigvals(int32_t p, const double *A, double *eig);
/* d = lambda_1(A) * (1 + 1e-10). */
double oracle_oem_d(int32_t p, const double *A);

/* ---- thresholding operators (Section 2.2, eqs. lasso, net, mcp, scad, glasso) ----
 * Scalar update for one coordinate: lam_w = w_j * lambda. */
double oracle_prox1(const oracle_penalty *pen, double u, double lam_w, double d);
/* Group lasso update of one group of length m: out = (u/d)(1 - lam_c/||u||)_+ */
void oracle_prox_group(int32_t m, const double *u, double lam_c, double d, double *out);
/* Update of one group of length m for any group penalty (Section 2.2, eqs.
 * glasso, gmcp, gscad, sglasso): group weight cgk, variable weights w (m
 * values, NULL = 1), penalty level lambda.  Group MCP / SCAD scale u by the
 * scalar MCP / SCAD update of ||u|| at c_k lambda.  The sparse group lasso
 * soft-thresholds each u_j at w_j lambda tau (no division by d) and then
 * applies the group lasso update at c_k lambda (1 - tau) with the same d; the
 * printed form divides by d in the inner step and uses 1 in the outer one,
 * which is not the proximal map unless d = 1. */
void oracle_prox_group_pen(const oracle_penalty *pen, int32_t m, const double *u, const double *w,
                           double cgk, double lambda, double d, double *out);

/* ---- lambda sequence ----
 * lambda_max: smallest lambda at which the update maps beta = 0 to 0 (tested
 * with the update's own arithmetic); lambda_l = lambda_max * ratio^(l/(L-1)). */
double oracle_lambda_max(int32_t p, const double *cs, const oracle_penalty *pen,
                         const int32_t *groups, int32_t ngroups, const double *w,
                         const double *cg);
void oracle_lambda_grid(double lambda_max, int32_t L, double ratio, double *lambda);

/* ---- OEM path (Section 2.1 update u = X^T y + A beta, A = d I - X^T X) ----
 * For each lambda in order, warm-started from the previous solution (beta = 0
 * before the first): repeat u = cs + d beta - Gs beta; beta <- prox(u)
 * until max|delta| <= tol * max|beta| or maxit updates.  groups: group id per
 * variable (0..ngroups-1), any partition; w (p) and cg (ngroups) nullable =
 * 1 and sqrt(|g|).  Outputs per lambda: beta (L x p), iteration count
 * (negated when maxit was reached), KKT violation, objective.
 * Returns 0, 1 if some lambda did not converge, < 0 on invalid input. */
int oracle_fit_path(int32_t p, const double *Gs, const double *cs, double yyn, double d,
                    const oracle_penalty *pen, const int32_t *groups, int32_t ngroups,
                    const double *w, const double *cg, int32_t L, const double *lambda,
                    double tol, int32_t maxit, double *beta, int32_t *iters, double *kkt,
                    double *obj);

/* Exactly nsteps OEM updates at one lambda from beta (in/out); objective
 * after each step into obj_trace (nsteps). */
int oracle_oem_steps(int32_t p, const double *Gs, const double *cs, double yyn, double d,
                     const oracle_penalty *pen, const int32_t *groups, int32_t ngroups,
                     const double *w, const double *cg, double lambda, int32_t nsteps,
                     double *beta, double *obj_trace);

/* Objective f and KKT violation of beta at lambda (standardised problem). */
double oracle_objective(int32_t p, const double *Gs, const double *cs, double yyn,
                        const oracle_penalty *pen, const int32_t *groups, int32_t ngroups,
                        const double *w, const double *cg, double lambda, const double *beta);
double oracle_kkt(int32_t p, const double *Gs, const double *cs, const oracle_penalty *pen,
                  const int32_t *groups, int32_t ngroups, const double *w, const double *cg,
                  double lambda, const double *beta);

/* ---- cross validation (Section 3; outputs of Section 5.5) ----
 * Held-out mean squared error of fold k computed row by row:
 * mse[l] = sum_{i in k} (y_i - beta0_l - x_i^T beta_l)^2 / n_k, beta on
 * original scale; beta0 (L intercepts) may be NULL (no intercept). */
int oracle_heldout_mse(const void *X, int32_t x_is_f64, int64_t n, int64_t ldx, int32_t p,
                       const double *y, int64_t row_offset, int32_t K, uint64_t fold_seed,
                       const uint8_t *foldid, int32_t k, int32_t L, const double *beta,
                       const double *beta0, double *mse);

/* ---- penalised logistic regression (Section 4) ----
 * y in {0, 1}, Pr(y = 1 | x) = 1 / (1 + exp(-x^T beta)), no intercept;
 * minimise (1/n) sum_i [log(1 + exp(x_i^T beta)) - y_i x_i^T beta] +
 * P_lambda(beta) (the printed log-likelihood's signs read as the standard
 * ones).  Proximal Newton with OEM as the inner solver: at the current
 * beta, w_i = mu_i (1 - mu_i) (hessian_bound: 1/4 for every i) and
 * z_i = x_i^T beta + (y_i - mu_i) / w_i; the quadratic model
 * (1/2n) sum w_i (z_i - x_i^T beta)^2 + P_lambda(beta) is minimised by OEM
 * updates (tol, maxit) from the current point on the standardised weighted
 * Gram with d = lambda_1 (1 + 1e-10); Newton steps repeat until max|delta
 * beta| <= newton_tol max|beta|.  Columns are standardised once, to unit
 * mean square.  Warm starts along lambda.  Outputs per lambda: beta (L x p,
 * original scale), Newton steps (negated at newton_maxit), the logistic
 * problem's stationarity violation and objective.  Returns 0, 1 when some
 * lambda hit newton_maxit, < 0 on bad input. */
int oracle_logistic_path(const void *X, int32_t x_is_f64, int64_t n, int64_t ldx, int32_t p,
                         const double *y, const oracle_penalty *pen, const int32_t *groups,
                         int32_t ngroups, const double *w, const double *cg, int32_t L,
                         const double *lambda, int32_t hessian_bound, double tol, int32_t maxit,
                         double newton_tol, int32_t newton_maxit, double *beta, int32_t *newton_iters,
                         double *kkt, double *obj);
/* lambda_max of that path: the penalty's zero level for c = X~^T (y - 1/2)/n. */
double oracle_logistic_lambda_max(const void *X, int32_t x_is_f64, int64_t n, int64_t ldx, int32_t p,
                                  const double *y, const oracle_penalty *pen, const int32_t *groups,
                                  int32_t ngroups, const double *w, const double *cg);

#ifdef __cplusplus
}
#endif
#endif
