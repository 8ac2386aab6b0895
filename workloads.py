"""Seeded synthetic inputs shaped like the paper's tall-data simulations.

This module only draws random numbers: it holds none of the OEM method's
arithmetic (no Gram, no thresholding, no fold assignment).  Both the CPU
oracle's tests and the GPU library's tests / benchmark take their inputs from
here, so the two implementations see identical bytes.

Workload shapes follow the paper's simulation designs: rows drawn from
N(0, Sigma) with AR(1) correlation Sigma_ij = rho^|i-j| (Section 6.1) or
compound symmetry (Section 5.2), a sparse true coefficient vector and Gaussian
noise.  The five named workloads are:

* ``small_lasso``      n=10,000  p=20   iid N(0,1), X stored FP64
* ``tall_multi``       n=1e6     p=100  AR(1) rho=0.5, X stored FP32
* ``cv_grouped``       n=2e6     p=500  AR(1) rho=0.3, FP32, 50 groups of 10
* ``batched_uneven``   64 problems, p log-uniform in [16, 2048], n=200 p
* ``serving``          request stream with Poisson arrivals

Every generator takes a ``scale`` (row-count multiplier) or explicit sizes so
tests can draw the same distributions at sizes the oracle finishes quickly.
"""
from __future__ import annotations

import math
import os
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

MASTER_SEED = 180109661
CHUNK_ROWS = 1 << 16


def subseed(*tags: int) -> np.random.SeedSequence:
    """Child seed sequence for a tuple of integer tags under the master seed."""
    return np.random.SeedSequence([MASTER_SEED, *[int(t) for t in tags]])


def _rng(ss: np.random.SeedSequence) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(ss))


def _threads() -> int:
    return max(1, min(16, os.cpu_count() or 1))


def draw_rows(n: int, p: int, rho: float, dtype, ss: np.random.SeedSequence,
              col_scale: Optional[np.ndarray] = None,
              correlation: str = "ar1") -> np.ndarray:
    """n x p row-major matrix with N(0, Sigma) rows, stored as ``dtype``.

    AR(1): x_j = rho x_{j-1} + sqrt(1-rho^2) z_j gives Sigma_ij = rho^|i-j|
    exactly.  Compound symmetry: x_j = sqrt(rho) z_0 + sqrt(1-rho) z_j gives
    Sigma_ij = rho (i != j), 1 on the diagonal.  Draws are FP64 and rounded
    once to ``dtype``.  Rows are generated in fixed 65536-row chunks, each from
    its own child seed, so the result does not depend on the thread count.
    """
    out = np.empty((n, p), dtype=dtype)
    nchunks = (n + CHUNK_ROWS - 1) // CHUNK_ROWS
    children = ss.spawn(nchunks) if nchunks else []
    sq = math.sqrt(max(0.0, 1.0 - rho * rho))

    def work(c: int) -> None:
        r0 = c * CHUNK_ROWS
        r1 = min(n, r0 + CHUNK_ROWS)
        g = _rng(children[c])
        z = g.standard_normal((r1 - r0, p))
        if correlation == "ar1" and rho != 0.0:
            for j in range(1, p):
                z[:, j] = rho * z[:, j - 1] + sq * z[:, j]
        elif correlation == "cs" and rho != 0.0:
            z0 = g.standard_normal((r1 - r0, 1))
            z = math.sqrt(rho) * z0 + math.sqrt(1.0 - rho) * z
        if col_scale is not None:
            z *= col_scale[None, :]
        out[r0:r1] = z

    if nchunks <= 1:
        for c in range(nchunks):
            work(c)
    else:
        with ThreadPoolExecutor(_threads()) as ex:
            list(ex.map(work, range(nchunks)))
    return out


def sparse_beta(p: int, k: int, ss: np.random.SeedSequence,
                positions: Optional[np.ndarray] = None) -> np.ndarray:
    """k nonzeros with random sign times U(0.5, 2) magnitude at seeded positions."""
    g = _rng(ss)
    beta = np.zeros(p)
    if positions is None:
        positions = np.sort(g.choice(p, size=k, replace=False))
    mags = g.uniform(0.5, 2.0, size=len(positions))
    signs = np.where(g.random(len(positions)) < 0.5, -1.0, 1.0)
    beta[positions] = signs * mags
    return beta


def response(X: np.ndarray, beta: np.ndarray, sigma: float,
             ss: np.random.SeedSequence) -> np.ndarray:
    """y = X beta + sigma * eps in FP64 from the stored (possibly FP32) X."""
    n = X.shape[0]
    g = _rng(ss)
    eps = g.standard_normal(n)
    y = np.empty(n)
    for r0 in range(0, n, CHUNK_ROWS):
        r1 = min(n, r0 + CHUNK_ROWS)
        y[r0:r1] = X[r0:r1].astype(np.float64) @ beta
    y += sigma * eps
    return y


@dataclass
class Problem:
    X: np.ndarray
    y: np.ndarray
    beta_true: np.ndarray
    rho: float
    groups: Optional[np.ndarray] = None
    col_scale: Optional[np.ndarray] = None
    meta: dict = field(default_factory=dict)


def small_lasso(n: int = 10_000, p: int = 20, seed_tag: int = 1) -> Problem:
    """n=1e4, p=20, iid N(0,1) FP64 X, 5 nonzeros, unit noise."""
    X = draw_rows(n, p, 0.0, np.float64, subseed(seed_tag, 0))
    b = sparse_beta(p, min(5, p), subseed(seed_tag, 1))
    y = response(X, b, 1.0, subseed(seed_tag, 2))
    return Problem(X, y, b, 0.0, meta=dict(workload="small_lasso", n=n, p=p))


def tall_multi(n: int = 1_000_000, p: int = 100, seed_tag: int = 2) -> Problem:
    """n=1e6, p=100, AR(1) rho=0.5 FP32 X, 10 nonzeros, unit noise."""
    X = draw_rows(n, p, 0.5, np.float32, subseed(seed_tag, 0))
    b = sparse_beta(p, min(10, p), subseed(seed_tag, 1))
    y = response(X, b, 1.0, subseed(seed_tag, 2))
    return Problem(X, y, b, 0.5, meta=dict(workload="tall_multi", n=n, p=p))


def cv_grouped(n: int = 2_000_000, p: int = 500, group_size: int = 10,
               active_groups: int = 5, seed_tag: int = 3, rho: float = 0.3) -> Problem:
    """n=2e6, p=500, AR(1) rho=0.3 FP32 X, contiguous groups, sigma=2."""
    X = draw_rows(n, p, rho, np.float32, subseed(seed_tag, 0))
    ngroups = (p + group_size - 1) // group_size
    groups = np.arange(p) // group_size
    g = _rng(subseed(seed_tag, 3))
    act = np.sort(g.choice(ngroups, size=min(active_groups, ngroups), replace=False))
    pos = np.concatenate([np.arange(a * group_size, min(p, (a + 1) * group_size)) for a in act])
    b = sparse_beta(p, len(pos), subseed(seed_tag, 1), positions=pos)
    y = response(X, b, 2.0, subseed(seed_tag, 2))
    return Problem(X, y, b, rho, groups=groups.astype(np.int32),
                   meta=dict(workload="cv_grouped", n=n, p=p))


def batched_uneven_shapes(nprob: int = 64, p_lo: int = 16, p_hi: int = 2048,
                          rows_per_col: int = 200, seed_tag: int = 4) -> List[tuple]:
    """(n, p) of each problem: p log-uniform in [p_lo, p_hi], n = rows_per_col * p."""
    g = _rng(subseed(seed_tag, 99))
    ps = np.rint(np.exp(g.uniform(math.log(p_lo), math.log(p_hi), size=nprob))).astype(int)
    return [(int(rows_per_col * p), int(p)) for p in ps]


def batched_uneven_problem(i: int, n: int, p: int, seed_tag: int = 4) -> Problem:
    """Problem i: N(0,1) columns times log-uniform scales in [0.1, 10]."""
    g = _rng(subseed(seed_tag, 1000 + i, 0))
    s = np.exp(g.uniform(math.log(0.1), math.log(10.0), size=p))
    X = draw_rows(n, p, 0.0, np.float32, subseed(seed_tag, 1000 + i, 1), col_scale=s)
    k = int(math.ceil(0.05 * p))
    b = sparse_beta(p, k, subseed(seed_tag, 1000 + i, 2)) / s
    y = response(X, b, 1.0, subseed(seed_tag, 1000 + i, 3))
    return Problem(X, y, b, 0.0, col_scale=s,
                   meta=dict(workload="batched_uneven", index=i, n=n, p=p))


@dataclass
class Request:
    index: int
    arrival_s: float
    n: int
    p: int
    rho: float
    penalty: str          # "lasso" | "mcp" | "scad" | "grp_lasso"
    nfolds: int           # 1 = plain fit, 5 = CV
    fold_seed: int


def serving_requests(count: int = 2000, rate_per_s: float = 50.0,
                     p_lo: int = 10, p_hi: int = 1000,
                     n_lo: int = 10_000, n_hi: int = 1_000_000,
                     seed_tag: int = 5) -> List[Request]:
    """Poisson arrivals, log-uniform p and n, rho ~ U(0, 0.8), mixed penalties."""
    g = _rng(subseed(seed_tag, 0))
    gaps = g.exponential(1.0 / rate_per_s, size=count)
    t = np.cumsum(gaps) - gaps[0]
    ps = np.rint(np.exp(g.uniform(math.log(p_lo), math.log(p_hi), size=count))).astype(int)
    ns = np.rint(np.exp(g.uniform(math.log(n_lo), math.log(n_hi), size=count))).astype(int)
    ns = np.maximum(ns, 10 * ps)
    rhos = g.uniform(0.0, 0.8, size=count)
    pens = g.integers(0, 4, size=count)
    cv = g.random(count) < 0.2
    fseeds = g.integers(0, 2**63 - 1, size=count, dtype=np.int64)
    names = ["lasso", "mcp", "scad", "grp_lasso"]
    return [Request(i, float(t[i]), int(ns[i]), int(ps[i]), float(rhos[i]), names[int(pens[i])],
                    5 if cv[i] else 1, int(fseeds[i])) for i in range(count)]


def serving_problem(req: Request, seed_tag: int = 5) -> Problem:
    """Data of one serving request: AR(1) FP32 rows, 5% nonzeros, unit noise."""
    X = draw_rows(req.n, req.p, req.rho, np.float32, subseed(seed_tag, 10 + req.index, 0))
    k = int(math.ceil(0.05 * req.p))
    b = sparse_beta(req.p, k, subseed(seed_tag, 10 + req.index, 1))
    y = response(X, b, 1.0, subseed(seed_tag, 10 + req.index, 2))
    groups = (np.arange(req.p) // 5).astype(np.int32)
    return Problem(X, y, b, req.rho, groups=groups,
                   meta=dict(workload="serving", index=req.index, n=req.n, p=req.p))


# The serving benchmark cannot draw ~185 MB of fresh rows per request at 50
# requests/s, so requests take the first n rows and p columns of one of 8
# pre-drawn matrices, one per AR(1) correlation level (rho quantised to the
# centres 0.05, 0.15, ..., 0.75); each request keeps its own coefficients and
# noise.
def serving_bucket(rho: float) -> int:
    return min(7, int(rho / 0.1))


def serving_pool(n: int, p: int, bucket: int, seed_tag: int = 5) -> np.ndarray:
    return draw_rows(n, p, 0.05 + 0.1 * bucket, np.float32, subseed(seed_tag, 900 + bucket))


def serving_response(req: Request, X: np.ndarray, seed_tag: int = 5):
    """(y, beta) of request `req` on rows X (n x p, any row stride)."""
    k = int(math.ceil(0.05 * req.p))
    b = sparse_beta(req.p, k, subseed(seed_tag, 10 + req.index, 1))
    supp = np.flatnonzero(b)
    g = _rng(subseed(seed_tag, 10 + req.index, 2))
    y = X[:, supp].astype(np.float64) @ b[supp] + g.standard_normal(X.shape[0])
    return y, b


def logistic(n: int = 1_000_000, p: int = 100, rho: float = 0.5, k: int = 10, scale: float = 0.5,
             seed_tag: int = 9, dtype=np.float32) -> Problem:
    """Binary responses for the logistic model of Section 4: AR(1) rows, k
    nonzero coefficients +-U(0.5, 2) times `scale`, y_i ~ Bernoulli(1 / (1 +
    exp(-x_i^T beta))) from seeded uniforms."""
    X = draw_rows(n, p, rho, dtype, subseed(seed_tag, 0))
    b = sparse_beta(p, min(k, p), subseed(seed_tag, 1)) * scale
    eta = np.zeros(n)
    for r0 in range(0, n, CHUNK_ROWS):
        eta[r0:r0 + CHUNK_ROWS] = X[r0:r0 + CHUNK_ROWS].astype(np.float64) @ b
    u = _rng(subseed(seed_tag, 2)).random(n)
    y = (u < 1.0 / (1.0 + np.exp(-eta))).astype(np.float64)
    return Problem(X, y, b, rho, meta=dict(workload="logistic", n=n, p=p))


@dataclass
class SparseProblem:
    rowptr: np.ndarray     # n + 1 int64
    col: np.ndarray        # nnz int32
    val: np.ndarray        # nnz float64
    y: np.ndarray          # n float64
    p: int
    beta: np.ndarray


def sparse_rows(n: int = 100_000, p: int = 200, density: float = 0.01, seed_tag: int = 8,
                dtype=np.float64, integer: bool = False) -> SparseProblem:
    """Sparse design in compressed sparse row form, shaped like the paper's
    sparse example (Section 5.8): round(density n p) positions drawn uniformly
    without replacement, N(0, 1) values (integers in [-8, 8] with
    integer=True), 15 nonzero coefficients U(-0.25, 0.25), y = X beta +
    N(0, 3^2)."""
    g = _rng(subseed(seed_tag, n, p))
    nnz = int(round(density * n * p))
    flat = np.sort(g.choice(n * p, size=nnz, replace=False))
    rows, cols = flat // p, (flat % p).astype(np.int32)
    if integer:
        val = g.integers(-8, 9, size=nnz).astype(dtype)
    else:
        val = g.standard_normal(nnz).astype(dtype)
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(rowptr, rows + 1, 1)
    rowptr = np.cumsum(rowptr)
    beta = np.zeros(p)
    beta[:15] = g.uniform(-0.25, 0.25, size=15)
    xb = np.zeros(n)
    np.add.at(xb, rows, val.astype(np.float64) * beta[cols])
    y = xb + 3.0 * g.standard_normal(n)
    if integer:
        y = np.rint(y)
    return SparseProblem(rowptr, cols, val, y, p, beta)


def integer_rows(n: int, p: int, lo: int = -8, hi: int = 8, seed_tag: int = 6,
                 dtype=np.float32) -> np.ndarray:
    """Integer-valued X: every Gram product and partial sum is exact in FP32/BF16/FP64."""
    g = _rng(subseed(seed_tag, n, p))
    return g.integers(lo, hi + 1, size=(n, p)).astype(dtype)


def integer_response(n: int, lo: int = -8, hi: int = 8, seed_tag: int = 7) -> np.ndarray:
    g = _rng(subseed(seed_tag, n))
    return g.integers(lo, hi + 1, size=n).astype(np.float64)
