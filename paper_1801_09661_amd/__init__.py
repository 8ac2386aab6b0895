"""MI355X (gfx950) OEM library for penalized least squares on tall data.

Thin Python binding over the C ABI of ``liboem.so`` (declared in
``include/oem.h``): argument marshalling only.  Every step of the method (the
Gram pass, standardisation, d, lambda grids, OEM paths, CV error and
selection) runs in the library's HIP kernels.  PyTorch supplies device memory
and streams.  There is no CPU fallback: without the built library, or without
a GPU, every call raises.
"""
from __future__ import annotations

import atexit
import ctypes as C
import os
import sys
import weakref
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("OEM_LIBRARY", os.path.join(HERE, "liboem.so"))

OEM_OK, OEM_NOT_CONVERGED = 0, 1
OEM_E_INVAL, OEM_E_NOMEM, OEM_E_HIP, OEM_E_STATE = -1, -2, -3, -4
OEM_FP64, OEM_SPLIT_BF16, OEM_BF16 = 0, 1, 2
OEM_X_F32, OEM_X_F64 = 0, 1
OEM_LASSO, OEM_ENET, OEM_MCP, OEM_SCAD, OEM_GRP_LASSO = 0, 1, 2, 3, 4
OEM_GRP_MCP, OEM_GRP_SCAD, OEM_SGL = 5, 6, 7

PENALTY_KIND = {"lasso": OEM_LASSO, "enet": OEM_ENET, "elastic_net": OEM_ENET, "mcp": OEM_MCP,
                "scad": OEM_SCAD, "grp_lasso": OEM_GRP_LASSO, "group_lasso": OEM_GRP_LASSO,
                "grp_mcp": OEM_GRP_MCP, "grp_scad": OEM_GRP_SCAD, "sgl": OEM_SGL,
                "sparse_grp_lasso": OEM_SGL}
PRECISION = {"fp64": OEM_FP64, "split_bf16": OEM_SPLIT_BF16, "bf16": OEM_BF16}

EXPORTED = ["oem_gram_create", "oem_gram_free", "oem_gram_reset", "oem_gram", "oem_gram_import",
            "oem_gram_export", "oem_fit_path", "oem_cv", "oem_gram_autotune", "oem_batch_create",
            "oem_batch_run", "oem_batch_run_graph", "oem_batch_status", "oem_batch_free",
            "oem_server_create", "oem_server_submit", "oem_server_poll", "oem_server_drain",
            "oem_server_now", "oem_server_free", "oem_last_error", "oem_version", "oem_gram_noalloc",
            "oem_gram_host", "oem_gram_export_colsums", "oem_gram_csr",
            "oem_logistic_path"]


class OemError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"oem error {code}: {msg}")
        self.code = code


class oem_penalty(C.Structure):
    _fields_ = [("kind", C.c_int32), ("alpha", C.c_double), ("gamma", C.c_double),
                ("tau", C.c_double)]


class oem_logistic_opts(C.Structure):
    _fields_ = [("hessian_bound", C.c_int32), ("newton_tol", C.c_double), ("newton_maxit", C.c_int32)]


class oem_path_opts(C.Structure):
    _fields_ = [("nlambda", C.c_int32), ("lambda_min_ratio", C.c_double),
                ("lambda_", C.POINTER(C.c_double)), ("tol", C.c_double), ("maxit", C.c_int32),
                ("standardize", C.c_int32), ("groups", C.POINTER(C.c_int32)),
                ("w", C.POINTER(C.c_double)), ("cg", C.POINTER(C.c_double)),
                ("sync", C.c_int32), ("intercept", C.c_int32), ("beta0", C.c_void_p)]


class oem_problem(C.Structure):
    _fields_ = [("p", C.c_int32), ("n", C.c_int64), ("ldx", C.c_int64), ("X", C.c_void_p),
                ("y", C.c_void_p), ("beta", C.c_void_p), ("lambda_", C.c_void_p),
                ("iters", C.c_void_p), ("kkt", C.c_void_p), ("obj", C.c_void_p),
                ("nfolds", C.c_int32), ("fold_seed", C.c_uint64), ("groups", C.c_void_p),
                ("lambda_in", C.c_void_p), ("beta_folds", C.c_void_p), ("cvm", C.c_void_p),
                ("cvsd", C.c_void_p), ("i_min", C.c_void_p), ("i_1se", C.c_void_p),
                ("best", C.c_void_p)]


class oem_request(C.Structure):
    _fields_ = [("id", C.c_int64), ("p", C.c_int32), ("n", C.c_int64), ("ldx", C.c_int64),
                ("X", C.c_void_p), ("y", C.c_void_p), ("nfolds", C.c_int32), ("fold_seed", C.c_uint64),
                ("pen", oem_penalty), ("groups", C.c_void_p), ("beta", C.c_void_p),
                ("lambda_", C.c_void_p), ("cvm", C.c_void_p), ("i_min", C.c_void_p),
                ("t_arrival", C.c_double)]


class oem_completion(C.Structure):
    _fields_ = [("id", C.c_int64), ("status", C.c_int32), ("slot", C.c_int32),
                ("t_arrival", C.c_double), ("t_admit", C.c_double), ("t_done", C.c_double),
                ("bytes", C.c_int64)]


_lib = None


def load_library(path: str = LIB_PATH) -> C.CDLL:
    """Load liboem.so; raise if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise OemError(OEM_E_STATE, f"{path} is missing: build it with "
                                    "`python -c 'import __graft_entry__ as g; g.build()'`")
    L = C.CDLL(path)
    vp, dp, ip, i64p = C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_int32), C.POINTER(C.c_int64)
    L.oem_gram_create.restype = C.c_int
    L.oem_gram_create.argtypes = [C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_uint64,
                                  C.POINTER(C.c_void_p)]
    L.oem_gram_free.restype = None
    L.oem_gram_free.argtypes = [vp]
    L.oem_gram_reset.restype = C.c_int
    L.oem_gram_reset.argtypes = [vp, vp]
    L.oem_gram.restype = C.c_int
    L.oem_gram.argtypes = [vp, vp, C.c_int64, C.c_int64, vp, C.c_int64, vp, vp]
    L.oem_logistic_path.restype = C.c_int
    L.oem_logistic_path.argtypes = [vp, C.c_int32, C.c_int64, C.c_int64, C.c_int32, vp,
                                    C.POINTER(oem_penalty), C.c_int32, C.POINTER(oem_path_opts),
                                    C.POINTER(oem_logistic_opts), vp, vp, vp, vp, vp, vp]
    L.oem_gram_csr.restype = C.c_int
    L.oem_gram_csr.argtypes = [vp, vp, vp, vp, C.c_int64, C.c_int64, vp, C.c_int64, vp, vp]
    L.oem_gram_host.restype = C.c_int
    L.oem_gram_host.argtypes = [vp, vp, C.c_int64, C.c_int64, vp, C.c_int64, vp, C.c_int64, vp]
    L.oem_gram_noalloc.restype = C.c_int
    L.oem_gram_noalloc.argtypes = [vp, vp, C.c_int64, C.c_int64, vp, C.c_int64, vp, vp]
    L.oem_gram_import.restype = C.c_int
    L.oem_gram_import.argtypes = [vp, C.c_int32, vp, vp, C.c_double, C.c_int64, C.c_int32, vp]
    L.oem_gram_export.restype = C.c_int
    L.oem_gram_export.argtypes = [vp, vp, vp, vp, vp, vp]
    L.oem_gram_export_colsums.restype = C.c_int
    L.oem_gram_export_colsums.argtypes = [vp, vp, vp, vp]
    L.oem_fit_path.restype = C.c_int
    L.oem_fit_path.argtypes = [vp, C.c_int32, C.POINTER(oem_penalty), C.c_int32,
                               C.POINTER(oem_path_opts), vp, vp, vp, vp, vp, vp, vp]
    L.oem_cv.restype = C.c_int
    L.oem_cv.argtypes = [vp, C.POINTER(oem_penalty), C.c_int32, C.POINTER(oem_path_opts), vp, vp,
                         vp, vp, vp, vp, vp, vp, vp, vp]
    L.oem_gram_autotune.restype = C.c_int
    L.oem_gram_autotune.argtypes = [vp, vp, C.c_int64, C.c_int64, vp, vp]
    L.oem_batch_create.restype = C.c_int
    L.oem_batch_create.argtypes = [C.POINTER(oem_problem), C.c_int32, C.c_int32, C.c_int32,
                                   C.POINTER(oem_penalty), C.c_int32, C.POINTER(oem_path_opts),
                                   C.POINTER(C.c_void_p)]
    for name in ("oem_batch_run", "oem_batch_run_graph", "oem_batch_status"):
        getattr(L, name).restype = C.c_int
        getattr(L, name).argtypes = [vp, vp]
    L.oem_batch_free.restype = None
    L.oem_batch_free.argtypes = [vp]
    L.oem_server_create.restype = C.c_int
    L.oem_server_create.argtypes = [C.c_int32, C.c_int64, C.c_int32, C.POINTER(oem_path_opts),
                                    C.POINTER(C.c_void_p)]
    L.oem_server_submit.restype = C.c_int
    L.oem_server_submit.argtypes = [vp, C.POINTER(oem_request)]
    L.oem_server_poll.restype = C.c_int
    L.oem_server_poll.argtypes = [vp, C.POINTER(oem_completion), C.c_int32, C.POINTER(C.c_int32),
                                  C.c_int32]
    L.oem_server_drain.restype = C.c_int
    L.oem_server_drain.argtypes = [vp]
    L.oem_server_now.restype = C.c_double
    L.oem_server_now.argtypes = []
    L.oem_server_free.restype = None
    L.oem_server_free.argtypes = [vp]
    L.oem_last_error.restype = C.c_char_p
    L.oem_last_error.argtypes = []
    L.oem_version.restype = C.c_char_p
    L.oem_version.argtypes = []
    _lib = L
    return L


# Owning wrappers (Gram, Batch, Server) register here.  At interpreter exit
# every live one is closed while the HIP runtime is still whole (the
# library's free calls wait for the device); finalizers that run later,
# during interpreter shutdown, make no library call at all.
_live = weakref.WeakSet()


@atexit.register
def _close_live() -> None:
    for obj in list(_live):
        try:
            obj.close()
        except Exception:
            pass


def _finalize(obj, _sys=sys) -> None:
    try:
        if _sys.is_finalizing():
            return
        obj.close()
    except Exception:
        pass


def _check(rc: int, allow_not_converged: bool = True) -> int:
    if rc == OEM_OK or (rc == OEM_NOT_CONVERGED and allow_not_converged):
        return rc
    msg = load_library().oem_last_error().decode()
    raise OemError(rc, msg)


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise OemError(OEM_E_STATE, "no GPU: the OEM library runs on the GPU only")
    return torch


def _ptr(t) -> Optional[int]:
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


@dataclass
class Penalty:
    kind: str = "lasso"
    alpha: float = 1.0
    gamma: float = 3.0
    tau: float = 0.0      # sparse group lasso mixing

    def c(self) -> oem_penalty:
        return oem_penalty(PENALTY_KIND[self.kind], float(self.alpha), float(self.gamma),
                           float(self.tau))


def _penalties(pens: Sequence) -> list:
    out = []
    for p in pens:
        if isinstance(p, Penalty):
            out.append(p)
        elif isinstance(p, str):
            out.append(Penalty(p))
        else:
            out.append(Penalty(**p))
    return out


# ------------------------------------------------------------------ C-ABI names

def oem_gram_create(p: int, nfolds: int = 1, precision: int = OEM_FP64, x_dtype: int = OEM_X_F32,
                    fold_seed: int = 0) -> C.c_void_p:
    _torch()
    h = C.c_void_p()
    _check(load_library().oem_gram_create(p, nfolds, precision, x_dtype,
                                          C.c_uint64(fold_seed & (2**64 - 1)), C.byref(h)))
    return h


def oem_gram_free(h) -> None:
    if h:
        load_library().oem_gram_free(h)


def oem_gram_reset(h, stream=None) -> None:
    _check(load_library().oem_gram_reset(h, _stream(stream)))


def oem_gram(h, X, y, row_offset: int = 0, foldid=None, stream=None, noalloc: bool = False) -> None:
    """Accumulate the statistics of the rows of X (cuda, row-major) and y
    (noalloc: through oem_gram_noalloc, the entry point that allocates nothing)."""
    torch = _torch()
    if X.dim() != 2 or X.stride(1) != 1:
        raise OemError(OEM_E_INVAL, "X must be a 2-D tensor with unit column stride")
    if not (X.is_cuda and y.is_cuda and y.dtype == torch.float64 and y.is_contiguous()):
        raise OemError(OEM_E_INVAL, "X, y must be cuda tensors; y contiguous float64")
    if foldid is not None and not (foldid.is_cuda and foldid.dtype == torch.uint8):
        raise OemError(OEM_E_INVAL, "foldid must be a cuda uint8 tensor")
    fn = load_library().oem_gram_noalloc if noalloc else load_library().oem_gram
    _check(fn(h, _ptr(X), X.shape[0], X.stride(0), _ptr(y), row_offset, _ptr(foldid),
              _stream(stream)))


def oem_gram_import(h, fold: int, XtX, Xty, yty: float, n: int, scaled: bool = True,
                    stream=None) -> None:
    _check(load_library().oem_gram_import(h, fold, _ptr(XtX), _ptr(Xty), float(yty), int(n),
                                          int(scaled), _stream(stream)))


def oem_gram_export(h, p: int, nfolds: int, stream=None):
    torch = _torch()
    G = torch.empty((nfolds, p, p), dtype=torch.float64, device="cuda")
    b = torch.empty((nfolds, p), dtype=torch.float64, device="cuda")
    yy = torch.empty(nfolds, dtype=torch.float64, device="cuda")
    nk = torch.empty(nfolds, dtype=torch.int64, device="cuda")
    _check(load_library().oem_gram_export(h, _ptr(G), _ptr(b), _ptr(yy), _ptr(nk), _stream(stream)))
    return G, b, yy, nk


class _Opts:
    """Keeps the host arrays referenced by an oem_path_opts alive."""

    def __init__(self, nlambda, lambda_min_ratio, lambdas, tol, maxit, standardize, groups, w, cg,
                 sync, intercept=False, beta0=None):
        self.lam = None if lambdas is None else np.ascontiguousarray(lambdas, dtype=np.float64)
        self.groups = None if groups is None else np.ascontiguousarray(groups, dtype=np.int32)
        self.w = None if w is None else np.ascontiguousarray(w, dtype=np.float64)
        self.cg = None if cg is None else np.ascontiguousarray(cg, dtype=np.float64)
        dp = lambda a: None if a is None else a.ctypes.data_as(C.POINTER(C.c_double))
        self.c = oem_path_opts(int(nlambda), float(lambda_min_ratio), dp(self.lam), float(tol),
                               int(maxit), int(standardize),
                               None if self.groups is None else
                               self.groups.ctypes.data_as(C.POINTER(C.c_int32)),
                               dp(self.w), dp(self.cg), int(sync), int(bool(intercept)),
                               None if beta0 is None else beta0.data_ptr())


def oem_fit_path(h, p: int, penalties: Sequence, fold: int = -1, nlambda: int = 100,
                 lambda_min_ratio: float = 1e-3, lambdas=None, tol: float = 1e-10,
                 maxit: int = 100000, standardize: bool = True, groups=None, w=None, cg=None,
                 sync: bool = True, stream=None, intercept: bool = False) -> dict:
    """Warm-started OEM paths; returns cuda tensors and the status code
    (with intercept=True also beta0, npen x L)."""
    torch = _torch()
    pens = _penalties(penalties)
    npen = len(pens)
    arr = (oem_penalty * npen)(*[q.c() for q in pens])
    f64 = dict(dtype=torch.float64, device="cuda")
    beta0 = torch.empty((npen, nlambda), **f64) if intercept else None
    o = _Opts(nlambda, lambda_min_ratio, lambdas, tol, maxit, standardize, groups, w, cg, sync,
              intercept, beta0)
    beta = torch.empty((npen, nlambda, p), **f64)
    lam = torch.empty((npen, nlambda), **f64)
    iters = torch.empty((npen, nlambda), dtype=torch.int32, device="cuda")
    kkt = torch.empty((npen, nlambda), **f64)
    obj = torch.empty((npen, nlambda), **f64)
    d = torch.empty(1, **f64)
    rc = _check(load_library().oem_fit_path(h, fold, arr, npen, C.byref(o.c), _ptr(beta), _ptr(lam),
                                            _ptr(iters), _ptr(kkt), _ptr(obj), _ptr(d),
                                            _stream(stream)))
    return dict(beta=beta, lambda_=lam, iters=iters, kkt=kkt, obj=obj, d=d, status=rc, beta0=beta0)


def oem_cv(h, p: int, nfolds: int, penalties: Sequence, nlambda: int = 100,
           lambda_min_ratio: float = 1e-3, lambdas=None, tol: float = 1e-10, maxit: int = 100000,
           standardize: bool = True, groups=None, w=None, cg=None, sync: bool = True,
           stream=None, intercept: bool = False) -> dict:
    """K-fold cross validation from the fold statistics; cuda tensors out."""
    torch = _torch()
    pens = _penalties(penalties)
    npen = len(pens)
    arr = (oem_penalty * npen)(*[q.c() for q in pens])
    f64 = dict(dtype=torch.float64, device="cuda")
    beta0 = torch.empty((npen, nlambda), **f64) if intercept else None
    o = _Opts(nlambda, lambda_min_ratio, lambdas, tol, maxit, standardize, groups, w, cg, sync,
              intercept, beta0)
    i32 = dict(dtype=torch.int32, device="cuda")
    beta_full = torch.empty((npen, nlambda, p), **f64)
    beta_folds = torch.empty((nfolds, npen, nlambda, p), **f64)
    lam = torch.empty((npen, nlambda), **f64)
    cvm = torch.empty((npen, nlambda), **f64)
    cvsd = torch.empty((npen, nlambda), **f64)
    i_min = torch.empty(npen, **i32)
    i_1se = torch.empty(npen, **i32)
    best = torch.empty(1, **i32)
    iters = torch.empty((nfolds + 1, npen, nlambda), **i32)
    rc = _check(load_library().oem_cv(h, arr, npen, C.byref(o.c), _ptr(beta_full), _ptr(beta_folds),
                                      _ptr(lam), _ptr(cvm), _ptr(cvsd), _ptr(i_min), _ptr(i_1se),
                                      _ptr(best), _ptr(iters), _stream(stream)))
    return dict(beta=beta_full, beta_folds=beta_folds, lambda_=lam, cvm=cvm, cvsd=cvsd,
                i_min=i_min, i_1se=i_1se, best=best, iters=iters, status=rc, beta0=beta0)


# ------------------------------------------------------------------ convenience

def logistic_path(X, y, penalties, nlambda: int = 100, lambda_min_ratio: float = 1e-3, lambdas=None,
                  tol: float = 1e-10, maxit: int = 100000, groups=None, w=None, cg=None,
                  hessian_bound: bool = False, newton_tol: float = 1e-10, newton_maxit: int = 100,
                  stream=None) -> dict:
    """Penalised logistic regression paths (oem_logistic_path, Section 4) on
    cuda tensors X (n x p, row-major) and y (n, float64, values 0 / 1)."""
    torch = _torch()
    if X.dim() != 2 or X.stride(1) != 1 or not X.is_cuda:
        raise OemError(OEM_E_INVAL, "X must be a 2-D cuda tensor with unit column stride")
    if not (y.is_cuda and y.dtype == torch.float64 and y.is_contiguous()):
        raise OemError(OEM_E_INVAL, "y must be a contiguous float64 cuda tensor")
    n, p = X.shape
    pens = _penalties(penalties)
    npen = len(pens)
    arr = (oem_penalty * npen)(*[q.c() for q in pens])
    o = _Opts(nlambda, lambda_min_ratio, lambdas, tol, maxit, True, groups, w, cg, False)
    lo = oem_logistic_opts(int(bool(hessian_bound)), float(newton_tol), int(newton_maxit))
    f64 = dict(dtype=torch.float64, device="cuda")
    beta = torch.empty((npen, nlambda, p), **f64)
    lam = torch.empty((npen, nlambda), **f64)
    newton = torch.empty((npen, nlambda), dtype=torch.int32, device="cuda")
    kkt = torch.empty((npen, nlambda), **f64)
    obj = torch.empty((npen, nlambda), **f64)
    xd = OEM_X_F64 if X.dtype == torch.float64 else OEM_X_F32
    rc = _check(load_library().oem_logistic_path(_ptr(X), xd, n, X.stride(0), p, _ptr(y), arr, npen,
                                                 C.byref(o.c), C.byref(lo), _ptr(beta), _ptr(lam),
                                                 _ptr(newton), _ptr(kkt), _ptr(obj), _stream(stream)))
    return dict(beta=beta, lambda_=lam, newton=newton, kkt=kkt, obj=obj, status=rc)


class Gram:
    """Owning wrapper of a library handle (statistics of one data set)."""

    def __init__(self, p: int, nfolds: int = 1, precision: str = "fp64", x_dtype=None,
                 fold_seed: int = 0):
        torch = _torch()
        xd = OEM_X_F64 if x_dtype in (torch.float64, "f64", OEM_X_F64) else OEM_X_F32
        self.p, self.nfolds, self.precision = p, nfolds, precision
        self.h = oem_gram_create(p, nfolds, PRECISION[precision], xd, fold_seed)
        _live.add(self)

    def close(self):
        if getattr(self, "h", None):
            oem_gram_free(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self, _fin=_finalize):
        # bound at class creation: module globals may already be cleared
        # when this runs during interpreter shutdown
        _fin(self)

    def add(self, X, y, row_offset: int = 0, foldid=None, stream=None, noalloc: bool = False):
        oem_gram(self.h, X, y, row_offset, foldid, stream, noalloc)
        return self

    def add_csr(self, rowptr, colidx, values, y, row_offset: int = 0, foldid=None, stream=None):
        """Sparse rows in compressed sparse row form (cuda tensors: int64
        rowptr, int32 colidx, values of the handle's element type)."""
        torch = _torch()
        if not (rowptr.is_cuda and rowptr.dtype == torch.int64 and colidx.dtype == torch.int32
                and y.is_cuda and y.dtype == torch.float64):
            raise OemError(OEM_E_INVAL, "rowptr int64, colidx int32, y float64 cuda tensors expected")
        n = rowptr.numel() - 1
        _check(load_library().oem_gram_csr(self.h, _ptr(rowptr), _ptr(colidx), _ptr(values),
                                           values.numel(), n, _ptr(y), row_offset, _ptr(foldid),
                                           _stream(stream)))
        return self

    def add_host(self, X, y, chunk_rows: int, row_offset: int = 0, foldid=None, stream=None):
        """Out-of-core pass over host rows (numpy arrays, memory maps or pinned
        tensors) streamed in chunks of chunk_rows rows."""
        oem_gram_host(self.h, X, y, chunk_rows, row_offset, foldid, stream)
        return self

    def export(self, stream=None):
        return oem_gram_export(self.h, self.p, self.nfolds, stream)

    def export_colsums(self, stream=None):
        """(column sums nfolds x p, sums of y nfolds) as cuda tensors."""
        torch = _torch()
        cs = torch.empty((self.nfolds, self.p), dtype=torch.float64, device="cuda")
        ys = torch.empty(self.nfolds, dtype=torch.float64, device="cuda")
        _check(load_library().oem_gram_export_colsums(self.h, _ptr(cs), _ptr(ys), _stream(stream)))
        return cs, ys

    def fit_path(self, penalties, fold: int = -1, **kw) -> dict:
        return oem_fit_path(self.h, self.p, penalties, fold=fold, **kw)

    def cv(self, penalties, **kw) -> dict:
        return oem_cv(self.h, self.p, self.nfolds, penalties, **kw)


def fit(X, y, penalties, precision: str = "fp64", **kw) -> dict:
    """Gram pass then full-data paths (the oem() call of Section 5.1)."""
    with Gram(X.shape[1], 1, precision, X.dtype) as g:
        g.add(X, y)
        return g.fit_path(penalties, **kw)


def cv(X, y, nfolds: int, fold_seed: int, penalties, precision: str = "fp64", foldid=None,
       **kw) -> dict:
    """Gram pass with fold statistics then K-fold CV (xval.oem of Section 5.5)."""
    with Gram(X.shape[1], nfolds, precision, X.dtype, fold_seed) as g:
        g.add(X, y, foldid=foldid)
        return g.cv(penalties, **kw)


def _host_array(a, dtypes):
    """(pointer, shape, row stride in elements) of a host array: a numpy array
    or memory map, or a CPU (possibly pinned) torch tensor."""
    if hasattr(a, "data_ptr"):       # the library itself rejects device memory
        if str(a.dtype).replace("torch.", "") not in dtypes or a.stride(-1) != 1:
            raise OemError(OEM_E_INVAL, "unsupported host tensor")
        return a.data_ptr(), tuple(a.shape), (a.stride(0) if a.dim() == 2 else 1)
    import numpy as np
    if a.dtype.name not in dtypes or a.strides[-1] != a.itemsize:
        raise OemError(OEM_E_INVAL, "unsupported host array")
    return a.ctypes.data, a.shape, (a.strides[0] // a.itemsize if a.ndim == 2 else 1)


def oem_gram_host(h, X, y, chunk_rows: int, row_offset: int = 0, foldid=None, stream=None) -> None:
    """Out-of-core Gram pass over host-resident rows (oem_gram_host)."""
    xp, xs, ldx = _host_array(X, ("float32", "float64"))
    yp, ys, _ = _host_array(y, ("float64",))
    if ys[0] != xs[0]:
        raise OemError(OEM_E_INVAL, "X and y row counts differ")
    fp = None if foldid is None else C.c_void_p(_host_array(foldid, ("uint8",))[0])
    _check(load_library().oem_gram_host(h, C.c_void_p(xp), xs[0], ldx, C.c_void_p(yp), row_offset,
                                        fp, chunk_rows, _stream(stream)))


def oem_gram_autotune(h, X, y, stream=None) -> None:
    """Tune the Gram pass of this handle's shape on (X, y); clears the sums."""
    n, p = X.shape
    _check(load_library().oem_gram_autotune(h, _ptr(X), n, X.stride(0), _ptr(y), _stream(stream)))


class Batch:
    """Many independent problems of uneven p fitted together (oem_batch_*).

    ``problems`` is a list of (X, y) cuda tensors (X row-major, FP32 or FP64
    for all) or of dicts with keys X, y and optionally nfolds (>= 2: K-fold
    CV), fold_seed, groups (p ints) and lambdas (npen x nlambda values used
    instead of the grid).  Outputs are cuda tensors per problem, refreshed by
    run(); CV problems also get beta_folds, cvm, cvsd, i_min, i_1se and best,
    and their iters cover the full data and every fold."""

    def __init__(self, problems, penalties, precision: str = "fp64", nlambda: int = 100,
                 lambda_min_ratio: float = 1e-3, tol: float = 1e-10, maxit: int = 100000):
        torch = _torch()
        pens = _penalties(penalties)
        self.npen, self.nlambda = len(pens), nlambda
        self.pen_arr = (oem_penalty * len(pens))(*[q.c() for q in pens])
        self.opts = _Opts(nlambda, lambda_min_ratio, None, tol, maxit, True, None, None, None, False)
        f64 = dict(dtype=torch.float64, device="cuda")
        i32 = dict(dtype=torch.int32, device="cuda")
        probs = [pr if isinstance(pr, dict) else dict(X=pr[0], y=pr[1]) for pr in problems]
        self.inputs = [(pr["X"], pr["y"]) for pr in probs]     # keep the device memory alive
        xd = OEM_X_F64 if probs[0]["X"].dtype == torch.float64 else OEM_X_F32
        self.out = []
        self._host = []                                        # host arrays read by create
        recs = []
        for pr in probs:
            X, y = pr["X"], pr["y"]
            n, p = X.shape
            K = int(pr.get("nfolds", 0) or 0)
            nq = K + 1 if K >= 2 else 1
            o = dict(beta=torch.zeros((self.npen, nlambda, p), **f64),
                     lambda_=torch.zeros((self.npen, nlambda), **f64),
                     iters=torch.zeros((nq, self.npen, nlambda) if K >= 2 else (self.npen, nlambda), **i32),
                     kkt=torch.zeros((self.npen, nlambda), **f64),
                     obj=torch.zeros((self.npen, nlambda), **f64))
            if K >= 2:
                o.update(beta_folds=torch.zeros((K, self.npen, nlambda, p), **f64),
                         cvm=torch.zeros((self.npen, nlambda), **f64),
                         cvsd=torch.zeros((self.npen, nlambda), **f64),
                         i_min=torch.zeros(self.npen, **i32), i_1se=torch.zeros(self.npen, **i32),
                         best=torch.zeros(1, **i32))
            self.out.append(o)
            g = pr.get("groups")
            g = None if g is None else np.ascontiguousarray(g, dtype=np.int32)
            lam = pr.get("lambdas")
            lam = None if lam is None else np.ascontiguousarray(lam, dtype=np.float64)
            if lam is not None and lam.size != self.npen * nlambda:
                raise OemError(OEM_E_INVAL, "lambdas must hold npen x nlambda values")
            self._host.append((g, lam))
            dp = lambda t: t.data_ptr() if t is not None else None
            hp = lambda a: a.ctypes.data if a is not None else None
            recs.append(oem_problem(p, n, X.stride(0), X.data_ptr(), y.data_ptr(), o["beta"].data_ptr(),
                                    o["lambda_"].data_ptr(), o["iters"].data_ptr(), o["kkt"].data_ptr(),
                                    o["obj"].data_ptr(), K, int(pr.get("fold_seed", 0)) & (2**64 - 1),
                                    hp(g), hp(lam), dp(o.get("beta_folds")), dp(o.get("cvm")),
                                    dp(o.get("cvsd")), dp(o.get("i_min")), dp(o.get("i_1se")),
                                    dp(o.get("best"))))
        self.recs = (oem_problem * len(recs))(*recs)
        h = C.c_void_p()
        _check(load_library().oem_batch_create(self.recs, len(recs), PRECISION[precision], xd,
                                               self.pen_arr, self.npen, C.byref(self.opts.c),
                                               C.byref(h)))
        self.h = h
        _live.add(self)

    def run(self, graph: bool = False, stream=None) -> None:
        f = load_library().oem_batch_run_graph if graph else load_library().oem_batch_run
        _check(f(self.h, _stream(stream)))

    def status(self, stream=None) -> int:
        return _check(load_library().oem_batch_status(self.h, _stream(stream)))

    def close(self):
        if getattr(self, "h", None):
            load_library().oem_batch_free(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self, _fin=_finalize):
        # bound at class creation: module globals may already be cleared
        # when this runs during interpreter shutdown
        _fin(self)


class Server:
    """Request loop (oem_server_*): submit fit / CV requests, collect completions.

    A request's X (FP32) and y may be pinned host tensors (pin_memory=True)
    or cuda tensors; its outputs are host arrays returned with the
    completion.  The caller keeps the inputs alive until then (the server
    keeps a reference)."""

    def __init__(self, nslots: int = 4, device_bytes: int = 64 << 30, precision: str = "fp64",
                 nlambda: int = 100, lambda_min_ratio: float = 1e-3, tol: float = 1e-10,
                 maxit: int = 100000):
        self.nlambda = nlambda
        self.opts = _Opts(nlambda, lambda_min_ratio, None, tol, maxit, True, None, None, None, False)
        h = C.c_void_p()
        _check(load_library().oem_server_create(nslots, int(device_bytes), PRECISION[precision],
                                                C.byref(self.opts.c), C.byref(h)))
        self.h = h
        self.live = {}
        self.results = {}
        _live.add(self)

    @staticmethod
    def now() -> float:
        return load_library().oem_server_now()

    def submit(self, rid: int, X, y, penalty, nfolds: int = 1, fold_seed: int = 0, groups=None,
               t_arrival: float = -1.0) -> None:
        pen = _penalties([penalty])[0].c()
        n, p = X.shape
        L = self.nlambda
        out = dict(beta=np.zeros((L, p)), lambda_=np.zeros(L), cvm=np.zeros(L),
                   i_min=np.zeros(1, dtype=np.int32))
        g = None if groups is None else np.ascontiguousarray(groups, dtype=np.int32)
        dp = lambda a: a.ctypes.data
        req = oem_request(int(rid), p, n, X.stride(0), X.data_ptr(), y.data_ptr(), int(nfolds),
                          int(fold_seed), pen, None if g is None else dp(g), dp(out["beta"]),
                          dp(out["lambda_"]), dp(out["cvm"]), dp(out["i_min"]), float(t_arrival))
        self.live[int(rid)] = (X, y, g, out, req)
        _check(load_library().oem_server_submit(self.h, C.byref(req)))

    def poll(self, wait: bool = True, max_n: int = 256) -> list:
        buf = (oem_completion * max_n)()
        cnt = C.c_int32(0)
        _check(load_library().oem_server_poll(self.h, buf, max_n, C.byref(cnt), 1 if wait else 0))
        res = []
        for i in range(cnt.value):
            c = buf[i]
            X, y, g, out, req = self.live.pop(int(c.id))
            rec = dict(id=int(c.id), status=int(c.status), slot=int(c.slot), t_arrival=c.t_arrival,
                       t_admit=c.t_admit, t_done=c.t_done, bytes=int(c.bytes), **out)
            self.results[int(c.id)] = rec
            res.append(rec)
        return res

    def drain(self) -> list:
        _check(load_library().oem_server_drain(self.h))
        out = []
        while True:
            got = self.poll(wait=False)
            if not got:
                return out
            out.extend(got)

    def close(self):
        if getattr(self, "h", None):
            load_library().oem_server_free(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self, _fin=_finalize):
        # bound at class creation: module globals may already be cleared
        # when this runs during interpreter shutdown
        _fin(self)
