"""OEM oracle: plain FP64 CPU reference (ctypes over oem_oracle.c).

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg import this package.  It shares no code with the
GPU library (``paper_1801_09661_amd``) and never imports it.

The C routines are naive FP64 loops that follow the paper's definitions; this
module only marshals arrays and strings the steps together in the paper's
order:

1. fold ids (Section 3, random partition) by the SplitMix64 hash;
2. Gram sums by row loops, and each training Gram computed directly from its
   rows (Section 3);
3. standardisation to unit-norm columns (Section 2.1);
4. d = lambda_1 * (1 + 1e-10) from a cyclic Jacobi eigen-solve (Section 2.1);
5. lambda sequence from the full-data statistics;
6. OEM updates (Section 2.1) with the thresholding operators of Section 2.2;
7. KKT violation and objective;
8. CV error from held-out rows directly and model selection (Section 5.5
   outputs).
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import Dict, List, Optional, Sequence

import numpy as np

from . import build as _build

LASSO, ENET, MCP, SCAD, GRP_LASSO, GRP_MCP, GRP_SCAD, SGL = 0, 1, 2, 3, 4, 5, 6, 7
KIND = {"lasso": LASSO, "enet": ENET, "elastic_net": ENET, "mcp": MCP, "scad": SCAD,
        "grp_lasso": GRP_LASSO, "group_lasso": GRP_LASSO, "grp_mcp": GRP_MCP,
        "grp_scad": GRP_SCAD, "sgl": SGL, "sparse_grp_lasso": SGL}
GROUP_KINDS = ("grp_lasso", "group_lasso", "grp_mcp", "grp_scad", "sgl", "sparse_grp_lasso")


class _Pen(C.Structure):
    _fields_ = [("kind", C.c_int32), ("alpha", C.c_double), ("gamma", C.c_double),
                ("tau", C.c_double)]


@dataclass
class Penalty:
    kind: str = "lasso"
    alpha: float = 1.0
    gamma: float = 3.0
    tau: float = 0.0

    def c(self) -> _Pen:
        return _Pen(KIND[self.kind], float(self.alpha), float(self.gamma), float(self.tau))


_lib = None


def lib():
    global _lib
    if _lib is None:
        path = os.environ.get("OEM_ORACLE_LIB", _build.LIB)
        if path == _build.LIB and not os.path.exists(path):
            _build.build()
        L = C.CDLL(path)
        dp, ip, u8p, i64p = (C.POINTER(C.c_double), C.POINTER(C.c_int32),
                             C.POINTER(C.c_uint8), C.POINTER(C.c_int64))
        vp = C.c_void_p
        pp = C.POINTER(_Pen)
        L.oracle_splitmix64_next.restype = C.c_uint64
        L.oracle_splitmix64_next.argtypes = [C.POINTER(C.c_uint64)]
        L.oracle_fold_of_row.restype = C.c_int32
        L.oracle_fold_of_row.argtypes = [C.c_uint64, C.c_int64, C.c_int32]
        L.oracle_fold_ids.restype = None
        L.oracle_fold_ids.argtypes = [C.c_uint64, C.c_int64, C.c_int64, C.c_int32, u8p]
        L.oracle_gram_folds.restype = C.c_int
        L.oracle_gram_folds.argtypes = [vp, C.c_int32, C.c_int64, C.c_int64, C.c_int32, dp,
                                        C.c_int64, C.c_int32, C.c_uint64, u8p, dp, dp, dp, i64p]
        L.oracle_gram_csr.restype = C.c_int
        L.oracle_gram_csr.argtypes = [i64p, ip, dp, C.c_int64, C.c_int32, dp, C.c_int64, C.c_int32,
                                      C.c_uint64, u8p, dp, dp, dp, i64p]
        L.oracle_gram_train.restype = C.c_int
        L.oracle_gram_train.argtypes = [vp, C.c_int32, C.c_int64, C.c_int64, C.c_int32, dp,
                                        C.c_int64, C.c_int32, C.c_uint64, u8p, C.c_int32,
                                        dp, dp, dp, i64p]
        L.oracle_standardize.restype = None
        L.oracle_standardize.argtypes = [C.c_int32, dp, dp, dp, dp, dp]
        L.oracle_sym_eigvals.restype = C.c_int
        L.oracle_sym_eigvals.argtypes = [C.c_int32, dp, dp]
        L.oracle_oem_d.restype = C.c_double
        L.oracle_oem_d.argtypes = [C.c_int32, dp]
        L.oracle_prox1.restype = C.c_double
        L.oracle_prox1.argtypes = [pp, C.c_double, C.c_double, C.c_double]
        L.oracle_prox_group.restype = None
        L.oracle_prox_group.argtypes = [C.c_int32, dp, C.c_double, C.c_double, dp]
        L.oracle_prox_group_pen.restype = None
        L.oracle_prox_group_pen.argtypes = [pp, C.c_int32, dp, dp, C.c_double, C.c_double,
                                            C.c_double, dp]
        L.oracle_lambda_max.restype = C.c_double
        L.oracle_lambda_max.argtypes = [C.c_int32, dp, pp, ip, C.c_int32, dp, dp]
        L.oracle_lambda_grid.restype = None
        L.oracle_lambda_grid.argtypes = [C.c_double, C.c_int32, C.c_double, dp]
        L.oracle_fit_path.restype = C.c_int
        L.oracle_fit_path.argtypes = [C.c_int32, dp, dp, C.c_double, C.c_double, pp, ip,
                                      C.c_int32, dp, dp, C.c_int32, dp, C.c_double, C.c_int32,
                                      dp, ip, dp, dp]
        L.oracle_oem_steps.restype = C.c_int
        L.oracle_oem_steps.argtypes = [C.c_int32, dp, dp, C.c_double, C.c_double, pp, ip,
                                       C.c_int32, dp, dp, C.c_double, C.c_int32, dp, dp]
        L.oracle_objective.restype = C.c_double
        L.oracle_objective.argtypes = [C.c_int32, dp, dp, C.c_double, pp, ip, C.c_int32, dp,
                                       dp, C.c_double, dp]
        L.oracle_kkt.restype = C.c_double
        L.oracle_kkt.argtypes = [C.c_int32, dp, dp, pp, ip, C.c_int32, dp, dp, C.c_double, dp]
        L.oracle_heldout_mse.restype = C.c_int
        L.oracle_heldout_mse.argtypes = [vp, C.c_int32, C.c_int64, C.c_int64, C.c_int32, dp,
                                         C.c_int64, C.c_int32, C.c_uint64, u8p, C.c_int32,
                                         C.c_int32, dp, dp, dp]
        L.oracle_logistic_path.restype = C.c_int
        L.oracle_logistic_path.argtypes = [vp, C.c_int32, C.c_int64, C.c_int64, C.c_int32, dp, pp,
                                           ip, C.c_int32, dp, dp, C.c_int32, dp, C.c_int32,
                                           C.c_double, C.c_int32, C.c_double, C.c_int32, dp, ip,
                                           dp, dp]
        L.oracle_logistic_lambda_max.restype = C.c_double
        L.oracle_logistic_lambda_max.argtypes = [vp, C.c_int32, C.c_int64, C.c_int64, C.c_int32, dp,
                                                 pp, ip, C.c_int32, dp, dp]
        _lib = L
    return _lib


# ---------------------------------------------------------------- marshalling

def _d(a: Optional[np.ndarray]):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _i(a: Optional[np.ndarray]):
    if a is None:
        return None
    assert a.dtype == np.int32 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_int32))


def _u8(a: Optional[np.ndarray]):
    if a is None:
        return None
    assert a.dtype == np.uint8 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_uint8))


def _f64(a) -> Optional[np.ndarray]:
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


def _x(X: np.ndarray):
    if X.dtype not in (np.float32, np.float64):
        raise TypeError("X must be float32 or float64")
    if X.ndim != 2 or X.strides[1] != X.itemsize or X.strides[0] % X.itemsize:
        raise ValueError("X must be row-major with unit column stride")
    return C.c_void_p(X.ctypes.data), int(X.dtype == np.float64), X.strides[0] // X.itemsize


# ---------------------------------------------------------------- primitives

def splitmix64(seed: int, count: int) -> List[int]:
    st = C.c_uint64(seed & (2**64 - 1))
    return [int(lib().oracle_splitmix64_next(C.byref(st))) for _ in range(count)]


def fold_ids(seed: int, n: int, K: int, row_offset: int = 0) -> np.ndarray:
    out = np.empty(n, dtype=np.uint8)
    lib().oracle_fold_ids(C.c_uint64(seed & (2**64 - 1)), row_offset, n, K, _u8(out))
    return out


def gram_folds(X, y, K: int = 1, fold_seed: int = 0, foldid=None, row_offset: int = 0):
    """Un-normalised per-fold sums (G_k, b_k, yy_k, n_k)."""
    n, p = X.shape
    xp, isf64, ldx = _x(X)
    y = _f64(y)
    G = np.zeros((K, p, p)); b = np.zeros((K, p)); yy = np.zeros(K)
    nk = np.zeros(K, dtype=np.int64)
    fid = None if foldid is None else np.ascontiguousarray(foldid, dtype=np.uint8)
    rc = lib().oracle_gram_folds(xp, isf64, n, ldx, p, _d(y), row_offset, K,
                                 C.c_uint64(fold_seed & (2**64 - 1)), _u8(fid), _d(G), _d(b),
                                 _d(yy), nk.ctypes.data_as(C.POINTER(C.c_int64)))
    if rc != 0:
        raise ValueError("oracle_gram_folds rejected its input")
    return G, b, yy, nk


def gram_csr(rowptr, col, val, p: int, y, K: int = 1, fold_seed: int = 0, foldid=None,
             row_offset: int = 0):
    """Per-fold sums (G_k, b_k, yy_k, n_k) of sparse rows (CSR, FP64 values)."""
    rp = np.ascontiguousarray(rowptr, dtype=np.int64)
    ci = np.ascontiguousarray(col, dtype=np.int32)
    v = np.ascontiguousarray(val, dtype=np.float64)
    y = _f64(y)
    n = len(rp) - 1
    G = np.zeros((K, p, p)); b = np.zeros((K, p)); yy = np.zeros(K)
    nk = np.zeros(K, dtype=np.int64)
    fid = None if foldid is None else np.ascontiguousarray(foldid, dtype=np.uint8)
    i64 = C.POINTER(C.c_int64)
    rc = lib().oracle_gram_csr(rp.ctypes.data_as(i64), _i(ci), _d(v), n, p, _d(y), row_offset, K,
                               C.c_uint64(fold_seed & (2**64 - 1)), _u8(fid), _d(G), _d(b), _d(yy),
                               nk.ctypes.data_as(i64))
    if rc != 0:
        raise ValueError("oracle_gram_csr rejected its input")
    return G, b, yy, nk


def gram_train(X, y, k: int = -1, K: int = 1, fold_seed: int = 0, foldid=None,
               row_offset: int = 0):
    """Un-normalised sums over the training rows of fold k (k = -1: all rows)."""
    n, p = X.shape
    xp, isf64, ldx = _x(X)
    y = _f64(y)
    G = np.zeros((p, p)); b = np.zeros(p); yy = C.c_double(0.0); nt = C.c_int64(0)
    fid = None if foldid is None else np.ascontiguousarray(foldid, dtype=np.uint8)
    rc = lib().oracle_gram_train(xp, isf64, n, ldx, p, _d(y), row_offset, K,
                                 C.c_uint64(fold_seed & (2**64 - 1)), _u8(fid), k, _d(G), _d(b),
                                 C.byref(yy), C.byref(nt))
    if rc != 0:
        raise ValueError("oracle_gram_train rejected its input")
    return G, b, yy.value, nt.value


def standardize(G: np.ndarray, c: np.ndarray):
    p = G.shape[0]
    G = _f64(G); c = _f64(c)
    Gs = np.empty((p, p)); cs = np.empty(p); s = np.empty(p)
    lib().oracle_standardize(p, _d(G), _d(c), _d(Gs), _d(cs), _d(s))
    return Gs, cs, s


def eigvals(A: np.ndarray) -> np.ndarray:
    A = _f64(A)
    e = np.empty(A.shape[0])
    if lib().oracle_sym_eigvals(A.shape[0], _d(A), _d(e)) < 0:
        raise RuntimeError("Jacobi did not converge")
    return np.sort(e)[::-1]


def oem_d(A: np.ndarray) -> float:
    A = _f64(A)
    return float(lib().oracle_oem_d(A.shape[0], _d(A)))


def prox1(pen: Penalty, u: float, lam_w: float, d: float) -> float:
    pc = pen.c()
    return float(lib().oracle_prox1(C.byref(pc), u, lam_w, d))


def prox_group(u: np.ndarray, lam_c: float, d: float) -> np.ndarray:
    u = _f64(u)
    out = np.empty_like(u)
    lib().oracle_prox_group(len(u), _d(u), lam_c, d, _d(out))
    return out


def prox_group_pen(pen: Penalty, u: np.ndarray, cgk: float, lam: float, d: float,
                   w: Optional[np.ndarray] = None) -> np.ndarray:
    """Update of one group for any group penalty (group weight cgk, level lam)."""
    u = _f64(u)
    out = np.empty_like(u)
    pc = pen.c()
    lib().oracle_prox_group_pen(C.byref(pc), len(u), _d(u), _d(_f64(w)), float(cgk), float(lam),
                                float(d), _d(out))
    return out


def _groups(groups, p):
    if groups is None:
        return None, 0
    g = np.ascontiguousarray(groups, dtype=np.int32)
    return g, int(g.max()) + 1 if p else 0


def lambda_max(cs, pen: Penalty, groups=None, w=None, cg=None) -> float:
    cs = _f64(cs); p = len(cs)
    g, ng = _groups(groups, p)
    pc = pen.c()
    return float(lib().oracle_lambda_max(p, _d(cs), C.byref(pc), _i(g), ng, _d(_f64(w)),
                                         _d(_f64(cg))))


def lambda_grid(lmax: float, L: int, ratio: float) -> np.ndarray:
    out = np.empty(L)
    lib().oracle_lambda_grid(lmax, L, ratio, _d(out))
    return out


def fit_path_std(Gs, cs, yyn, d, pen: Penalty, lambdas, groups=None, w=None, cg=None,
                 tol=1e-10, maxit=100000):
    """OEM path on a standardised (or raw) Gram; returns dict of arrays."""
    Gs = _f64(Gs); cs = _f64(cs); lam = _f64(lambdas)
    p = len(cs); L = len(lam)
    g, ng = _groups(groups, p)
    beta = np.zeros((L, p)); it = np.zeros(L, dtype=np.int32); kkt = np.zeros(L)
    obj = np.zeros(L)
    pc = pen.c()
    rc = lib().oracle_fit_path(p, _d(Gs), _d(cs), float(yyn), float(d), C.byref(pc), _i(g), ng,
                               _d(_f64(w)), _d(_f64(cg)), L, _d(lam), tol, maxit, _d(beta),
                               _i(it), _d(kkt), _d(obj))
    if rc < 0:
        raise ValueError("oracle_fit_path rejected its input")
    return dict(beta_std=beta, iters=it, kkt=kkt, obj=obj, status=rc)


def oem_steps(Gs, cs, yyn, d, pen: Penalty, lam, beta0, nsteps, groups=None, w=None, cg=None):
    Gs = _f64(Gs); cs = _f64(cs)
    beta = np.array(beta0, dtype=np.float64, copy=True)
    p = len(cs)
    g, ng = _groups(groups, p)
    tr = np.zeros(nsteps)
    pc = pen.c()
    rc = lib().oracle_oem_steps(p, _d(Gs), _d(cs), float(yyn), float(d), C.byref(pc), _i(g), ng,
                                _d(_f64(w)), _d(_f64(cg)), float(lam), nsteps, _d(beta), _d(tr))
    if rc != 0:
        raise ValueError("oracle_oem_steps rejected its input")
    return beta, tr


def objective(Gs, cs, yyn, pen: Penalty, lam, beta, groups=None, w=None, cg=None) -> float:
    Gs = _f64(Gs); cs = _f64(cs); beta = _f64(beta)
    g, ng = _groups(groups, len(cs))
    pc = pen.c()
    return float(lib().oracle_objective(len(cs), _d(Gs), _d(cs), float(yyn), C.byref(pc), _i(g),
                                        ng, _d(_f64(w)), _d(_f64(cg)), float(lam), _d(beta)))


def kkt(Gs, cs, pen: Penalty, lam, beta, groups=None, w=None, cg=None) -> float:
    Gs = _f64(Gs); cs = _f64(cs); beta = _f64(beta)
    g, ng = _groups(groups, len(cs))
    pc = pen.c()
    return float(lib().oracle_kkt(len(cs), _d(Gs), _d(cs), C.byref(pc), _i(g), ng, _d(_f64(w)),
                                  _d(_f64(cg)), float(lam), _d(beta)))


def heldout_mse(X, y, k: int, K: int, fold_seed: int, beta_orig: np.ndarray, foldid=None,
                row_offset: int = 0, beta0=None) -> np.ndarray:
    n, p = X.shape
    xp, isf64, ldx = _x(X)
    y = _f64(y); b = _f64(beta_orig)
    L = b.shape[0]
    mse = np.zeros(L)
    fid = None if foldid is None else np.ascontiguousarray(foldid, dtype=np.uint8)
    rc = lib().oracle_heldout_mse(xp, isf64, n, ldx, p, _d(y), row_offset, K,
                                  C.c_uint64(fold_seed & (2**64 - 1)), _u8(fid), k, L, _d(b),
                                  _d(_f64(beta0)), _d(mse))
    if rc != 0:
        raise ValueError("oracle_heldout_mse: empty fold or bad input")
    return mse


# ---------------------------------------------------------------- pipelines

def _as_pen(p) -> Penalty:
    if isinstance(p, Penalty):
        return p
    if isinstance(p, str):
        return Penalty(p)
    return Penalty(**p)


def prepare(G_sum, b_sum, yy_sum, n, standardize_flag=True):
    """Scaled statistics (G/n, c/n, yy/n) and the standardised problem."""
    G = G_sum / n
    c = b_sum / n
    yyn = yy_sum / n
    if standardize_flag:
        Gs, cs, s = standardize(G, c)
    else:
        Gs, cs, s = G.copy(), c.copy(), np.ones(len(c))
    return dict(G=G, c=c, yyn=yyn, Gs=Gs, cs=cs, s=s)


def lambda_sequences(cs_full, penalties, nlambda=100, lambda_min_ratio=1e-3, groups=None, w=None,
                     cg=None) -> np.ndarray:
    out = np.zeros((len(penalties), nlambda))
    for i, pen in enumerate(penalties):
        pen = _as_pen(pen)
        out[i] = lambda_grid(lambda_max(cs_full, pen, groups, w, cg), nlambda, lambda_min_ratio)
    return out


def fit_from_stats(st: dict, penalties, lambdas: np.ndarray, groups=None, w=None, cg=None,
                   tol=1e-10, maxit=100000, d: Optional[float] = None) -> dict:
    d = oem_d(st["Gs"]) if d is None else d
    res = dict(d=d, beta_std=[], beta=[], iters=[], kkt=[], obj=[], status=0)
    for i, pen in enumerate(penalties):
        r = fit_path_std(st["Gs"], st["cs"], st["yyn"], d, _as_pen(pen), lambdas[i], groups, w, cg,
                         tol, maxit)
        res["beta_std"].append(r["beta_std"])
        res["beta"].append(r["beta_std"] / st["s"][None, :])
        res["iters"].append(r["iters"]); res["kkt"].append(r["kkt"]); res["obj"].append(r["obj"])
        res["status"] = max(res["status"], r["status"])
    for key in ("beta_std", "beta", "iters", "kkt", "obj"):
        res[key] = np.stack(res[key])
    res["lambda"] = lambdas
    return res


def centred(X, y, rows=None):
    """X and y in FP64 with the means of the selected rows (all rows when
    rows is None) subtracted: fitting an unpenalised intercept by its plain
    definition.  Returns (Xc, yc, xbar, ybar)."""
    X64 = np.asarray(X, dtype=np.float64)
    y64 = np.asarray(y, dtype=np.float64)
    sel = slice(None) if rows is None else rows
    xbar = X64[sel].mean(axis=0)
    ybar = float(y64[sel].mean())
    return np.ascontiguousarray(X64 - xbar), y64 - ybar, xbar, ybar


def fit(X, y, penalties: Sequence, groups=None, w=None, cg=None, nlambda=100,
        lambda_min_ratio=1e-3, lambdas=None, tol=1e-10, maxit=100000, standardize=True,
        intercept=False) -> dict:
    """Full-data OEM paths (the oem() call of Section 5.1).  intercept: the
    columns and y are centred first and beta0 = ybar - xbar^T beta."""
    penalties = [_as_pen(p) for p in penalties]
    if intercept:
        Xc, yc, xbar, ybar = centred(X, y)
        G, b, yy, n = gram_train(Xc, yc, -1)
    else:
        G, b, yy, n = gram_train(X, y, -1)
    st = prepare(G, b, yy, n, standardize)
    if lambdas is None:
        lambdas = lambda_sequences(st["cs"], penalties, nlambda, lambda_min_ratio, groups, w, cg)
    res = fit_from_stats(st, penalties, np.asarray(lambdas, dtype=np.float64), groups, w, cg, tol,
                         maxit)
    res["stats"] = st
    if intercept:
        res["beta0"] = ybar - res["beta"] @ xbar
        res["xbar"], res["ybar"] = xbar, ybar
    return res


def select(mse: np.ndarray, nk: np.ndarray) -> dict:
    """CV summaries from per-fold held-out MSE (npen x K x L)."""
    npen, K, L = mse.shape
    n = float(nk.sum())
    w = nk.astype(np.float64) / n
    cvm = np.einsum("k,pkl->pl", w, mse)
    dev = mse - cvm[:, None, :]
    cvsd = np.sqrt(np.einsum("k,pkl->pl", nk.astype(np.float64), dev * dev) / (n * (K - 1)))
    i_min = np.argmin(cvm, axis=1)
    i_1se = np.zeros(npen, dtype=np.int64)
    for q in range(npen):
        thr = cvm[q, i_min[q]] + cvsd[q, i_min[q]]
        i_1se[q] = int(np.nonzero(cvm[q] <= thr)[0][0])
    mins = cvm[np.arange(npen), i_min]
    best = int(np.argmin(mins))
    return dict(cvm=cvm, cvsd=cvsd, i_min=i_min, i_1se=i_1se, best=best)


def cv(X, y, K: int, fold_seed: int, penalties: Sequence, groups=None, w=None, cg=None,
       nlambda=100, lambda_min_ratio=1e-3, lambdas=None, tol=1e-10, maxit=100000,
       standardize=True, foldid=None, intercept=False) -> dict:
    """K-fold CV (Section 3): training Grams per fold, paths, held-out error.
    intercept: each fold's training rows are centred with their own means and
    its held-out residuals are y - beta0 - x^T beta."""
    penalties = [_as_pen(p) for p in penalties]
    full = fit(X, y, penalties, groups, w, cg, nlambda, lambda_min_ratio, lambdas, tol, maxit,
               standardize, intercept)
    lam = full["lambda"]
    folds = []
    mse = np.zeros((len(penalties), K, lam.shape[1]))
    nk = np.zeros(K, dtype=np.int64)
    fid = (np.ascontiguousarray(foldid, dtype=np.uint8) if foldid is not None
           else fold_ids(fold_seed, X.shape[0], K))
    for k in range(K):
        if intercept:
            Xc, yc, xbar, ybar = centred(X, y, fid != k)
            G, b, yy, nt = gram_train(Xc, yc, k, K, fold_seed, foldid)
        else:
            G, b, yy, nt = gram_train(X, y, k, K, fold_seed, foldid)
        st = prepare(G, b, yy, nt, standardize)
        r = fit_from_stats(st, penalties, lam, groups, w, cg, tol, maxit)
        if intercept:
            r["beta0"] = ybar - r["beta"] @ xbar
        for q in range(len(penalties)):
            mse[q, k] = heldout_mse(X, y, k, K, fold_seed, r["beta"][q], foldid,
                                    beta0=r["beta0"][q] if intercept else None)
        nk[k] = X.shape[0] - nt
        folds.append(r)
    sel = select(mse, nk)
    return dict(full=full, folds=folds, mse=mse, nk=nk, **sel)


def logistic_path(X, y, penalties: Sequence, groups=None, w=None, cg=None, nlambda=100,
                  lambda_min_ratio=1e-3, lambdas=None, hessian_bound=False, tol=1e-10,
                  maxit=100000, newton_tol=1e-10, newton_maxit=100) -> dict:
    """Penalised logistic regression paths (Section 4): proximal Newton with
    an OEM inner loop.  y in {0, 1}; no intercept."""
    penalties = [_as_pen(p) for p in penalties]
    n, p = X.shape
    xp, isf64, ldx = _x(X)
    y = _f64(y)
    g, ng = _groups(groups, p)
    if lambdas is None:
        lambdas = np.zeros((len(penalties), nlambda))
        for i, pen in enumerate(penalties):
            pc = pen.c()
            lm = float(lib().oracle_logistic_lambda_max(xp, isf64, n, ldx, p, _d(y), C.byref(pc),
                                                        _i(g), ng, _d(_f64(w)), _d(_f64(cg))))
            lambdas[i] = lambda_grid(lm, nlambda, lambda_min_ratio)
    lambdas = np.ascontiguousarray(lambdas, dtype=np.float64)
    L = lambdas.shape[1]
    out = dict(beta=np.zeros((len(penalties), L, p)), newton=np.zeros((len(penalties), L), np.int32),
               kkt=np.zeros((len(penalties), L)), obj=np.zeros((len(penalties), L)), lambda_=lambdas,
               status=0)
    for i, pen in enumerate(penalties):
        pc = pen.c()
        b = np.zeros((L, p)); it = np.zeros(L, dtype=np.int32); kk = np.zeros(L); ob = np.zeros(L)
        rc = lib().oracle_logistic_path(xp, isf64, n, ldx, p, _d(y), C.byref(pc), _i(g), ng,
                                        _d(_f64(w)), _d(_f64(cg)), L, _d(lambdas[i]),
                                        int(bool(hessian_bound)), tol, maxit, newton_tol,
                                        newton_maxit, _d(b), _i(it), _d(kk), _d(ob))
        if rc < 0:
            raise ValueError("oracle_logistic_path rejected its input")
        out["beta"][i], out["newton"][i], out["kkt"][i], out["obj"][i] = b, it, kk, ob
        out["status"] = max(out["status"], rc)
    return out
