"""GPU parity of the OEM paths and cross validation (FP64 form) against the
oracle.

Tolerance (coefficients, FP64): both sides stop when the last update moved
beta by at most tol * max|beta| (tol = 1e-10), from the same warm start, the
same d (to ~1e-12) and the same lambda grid; a stopping decision that differs
by one update moves beta by at most tol * max|beta|.  Hence, per (penalty,
lambda): max|beta_gpu - beta_oracle| <= 1e-10 * max|beta_oracle|.  Active sets
(nonzero patterns) must match exactly.
"""
import numpy as np
import pytest

import oracle
import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-10


def _oem():
    import paper_1801_09661_amd as oem
    return oem


def _cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _assert_paths(b_gpu, b_or, tol=TOL, skip_first=False, what=""):
    """b_*: (npen, L, p).  Per (penalty, lambda) relative inf-norm error."""
    for q in range(b_or.shape[0]):
        for l in range(b_or.shape[1]):
            ref = b_or[q, l]
            got = b_gpu[q, l]
            scale = np.abs(ref).max()
            if scale == 0.0:
                assert np.all(got == 0.0), f"{what} pen {q} lambda {l}: expected all-zero"
                continue
            err = np.abs(got - ref).max() / scale
            assert err <= tol, f"{what} pen {q} lambda {l}: rel err {err:.3e}"
            assert np.array_equal(got != 0, ref != 0), f"{what} pen {q} lambda {l}: active set"


def _fit_both(pr, pens, L, ratio=1e-3, groups=None, **kw):
    oem = _oem()
    res = oem.fit(_cuda(pr.X), _cuda(pr.y), pens, nlambda=L, lambda_min_ratio=ratio, tol=TOL,
                  groups=groups, **kw)
    torch.cuda.synchronize()
    ref = oracle.fit(pr.X, pr.y, pens, groups=groups, nlambda=L, lambda_min_ratio=ratio, tol=TOL,
                     **{k: v for k, v in kw.items() if k in ("w", "cg", "standardize", "maxit")})
    return res, ref


def test_small_lasso_workload_parity():
    """n=1e4, p=20, iid FP64 X, lasso, 50 lambdas, tol 1e-10 (full size)."""
    print("case: small_lasso full size", flush=True)
    pr = workloads.small_lasso()
    res, ref = _fit_both(pr, ["lasso"], 50)
    d = res["d"].item()
    assert abs(d - ref["d"]) <= 1e-12 * ref["d"]
    lam = res["lambda_"].cpu().numpy()
    assert np.allclose(lam, ref["lambda"], rtol=1e-14, atol=0)
    _assert_paths(res["beta"].cpu().numpy(), ref["beta"], what="lasso")
    it = res["iters"].cpu().numpy()
    assert np.all(it > 0)
    assert np.all(np.abs(it - ref["iters"]) <= 1)
    assert np.allclose(res["obj"].cpu().numpy(), ref["obj"], rtol=1e-12)


@pytest.mark.parametrize("p", [1, 2, 30, 32, 33, 64, 65, 128, 150, 513])
def test_four_penalties_parity(p):
    n = 20_000 if p <= 200 else 12_000
    print(f"case: tall_multi scaled n={n} p={p}", flush=True)
    pr = workloads.tall_multi(n=n, p=p, seed_tag=200 + p)
    pens = [dict(kind="lasso"), dict(kind="enet", alpha=0.5), dict(kind="mcp", gamma=3.0),
            dict(kind="scad", gamma=3.7)]
    res, ref = _fit_both(pr, pens, 30)
    _assert_paths(res["beta"].cpu().numpy(), ref["beta"], what=f"p={p}")
    k = res["kkt"].cpu().numpy()
    assert np.all(k <= 1e-8)


def test_group_lasso_parity_noncontiguous_groups():
    print("case: group lasso, shuffled group ids", flush=True)
    pr = workloads.cv_grouped(n=20_000, p=40, group_size=5, active_groups=3, seed_tag=210)
    rng = np.random.default_rng(0)
    groups = rng.permutation(pr.groups).astype(np.int32)
    res, ref = _fit_both(pr, ["grp_lasso"], 25, groups=groups)
    _assert_paths(res["beta"].cpu().numpy(), ref["beta"], what="grp")


def test_group_lasso_parity_large_p_noncontiguous():
    """p = 300 (streaming kernel), shuffled group ids of size 10."""
    print("case: group lasso p=300, shuffled group ids", flush=True)
    pr = workloads.cv_grouped(n=15_000, p=300, group_size=10, active_groups=4, seed_tag=217)
    rng = np.random.default_rng(1)
    groups = rng.permutation(pr.groups).astype(np.int32)
    res, ref = _fit_both(pr, ["grp_lasso", "lasso"], 20, groups=groups)
    _assert_paths(res["beta"].cpu().numpy(), ref["beta"], what="grp p=300")
    assert np.all(res["kkt"].cpu().numpy() <= 1e-8)


def test_weights_and_unstandardized():
    print("case: weights + standardize=0", flush=True)
    pr = workloads.small_lasso(n=5000, p=12, seed_tag=211)
    w = np.linspace(0.5, 2.0, 12)
    res, ref = _fit_both(pr, ["lasso", dict(kind="mcp", gamma=4.0)], 20, w=w, standardize=False)
    _assert_paths(res["beta"].cpu().numpy(), ref["beta"], what="weighted")


def test_zero_column_unstandardized():
    """A column of zeros (standardize=0): its coefficient stays zero and its
    screening key is unbounded, which must neither stall nor shift the rest."""
    print("case: zero column, standardize=0, p=70", flush=True)
    pr = workloads.tall_multi(n=6000, p=70, seed_tag=219)
    pr.X[:, 7] = 0.0
    pr.X[:, 41] = 0.0
    res, ref = _fit_both(pr, ["lasso", dict(kind="scad", gamma=3.7)], 25, standardize=False)
    b = res["beta"].cpu().numpy()
    assert np.all(b[:, :, 7] == 0.0) and np.all(b[:, :, 41] == 0.0)
    _assert_paths(b, ref["beta"], what="zero column")


@pytest.mark.parametrize("p,n", [(48, 400), (100, 600), (120, 300_000), (260, 2_000)])
def test_active_set_outgrows_working_set(p, n):
    """Short, wide-ish problems whose active sets outgrow 32, 64 and 128
    coordinates part-way along the path, so every path is handed from one
    kernel to the next at some lambda (mid-lambda and at lambda ends).
    Parity over the whole path."""
    print(f"case: working-set hand-over p={p} n={n}", flush=True)
    pr = workloads.tall_multi(n=n, p=p, seed_tag=230 + p)
    pens = [dict(kind="lasso"), dict(kind="enet", alpha=0.5), dict(kind="mcp", gamma=3.0),
            dict(kind="scad", gamma=3.7)]
    res, ref = _fit_both(pr, pens, 40, ratio=1e-4)
    _assert_paths(res["beta"].cpu().numpy(), ref["beta"], what=f"hand-over p={p}")
    it = res["iters"].cpu().numpy()
    assert np.all(it > 0)
    assert np.all(np.abs(it - ref["iters"]) <= 1)
    assert np.all(res["kkt"].cpu().numpy() <= 1e-8)


def test_group_active_set_outgrows_working_set():
    """Group lasso whose active groups outgrow the working set (p=150,
    groups of 7 and 3, n small)."""
    print("case: group working-set hand-over p=150", flush=True)
    pr = workloads.tall_multi(n=700, p=150, seed_tag=241)
    groups = np.repeat(np.arange(30), [7, 3] * 15).astype(np.int32)
    rng = np.random.default_rng(5)
    groups = rng.permutation(groups)
    res, ref = _fit_both(pr, ["grp_lasso"], 30, ratio=1e-4, groups=groups)
    _assert_paths(res["beta"].cpu().numpy(), ref["beta"], what="grp hand-over")
    assert np.all(res["kkt"].cpu().numpy() <= 1e-8)


def test_explicit_lambda_and_lambda_zero():
    oem = _oem()
    pr = workloads.tall_multi(n=8000, p=10, seed_tag=212)
    lam = np.array([[0.2, 0.05, 0.0]])
    res = oem.fit(_cuda(pr.X), _cuda(pr.y), ["lasso"], nlambda=3, lambdas=lam, tol=1e-13)
    ref = oracle.fit(pr.X, pr.y, ["lasso"], lambdas=lam, tol=1e-13)
    _assert_paths(res["beta"].cpu().numpy(), ref["beta"], tol=1e-12, what="explicit")
    ols = np.linalg.lstsq(pr.X.astype(np.float64), pr.y, rcond=None)[0]
    assert np.abs(res["beta"].cpu().numpy()[0, 2] - ols).max() <= 1e-8 * np.abs(ols).max()


def test_maxit_reports_nonconvergence():
    oem = _oem()
    pr = workloads.tall_multi(n=8000, p=10, seed_tag=213)
    res = oem.fit(_cuda(pr.X), _cuda(pr.y), ["lasso"], nlambda=5, maxit=2)
    assert res["status"] == oem.OEM_NOT_CONVERGED
    it = res["iters"].cpu().numpy()[0]
    assert it[0] == 1 and np.all(it[1:] == -2)


def test_invalid_inputs_raise():
    oem = _oem()
    pr = workloads.small_lasso(n=500, p=5, seed_tag=214)
    X, y = _cuda(pr.X), _cuda(pr.y)
    with pytest.raises(oem.OemError):
        oem.fit(X, y, [dict(kind="mcp", gamma=0.5)], nlambda=3)
    with pytest.raises(oem.OemError):
        oem.fit(X, y, ["grp_lasso"], nlambda=3)          # no groups
    with pytest.raises(oem.OemError):
        oem.fit(X, y, [dict(kind="enet", alpha=0.0)], nlambda=3)
    with oem.Gram(5, 1, "fp64", X.dtype) as g:
        with pytest.raises(oem.OemError):
            g.fit_path(["lasso"], nlambda=3)             # no rows yet


def test_cv_parity_grouped_workload_scaled():
    """Scaled-down CV workload: K=5 hashed folds, group lasso + lasso + MCP."""
    oem = _oem()
    K, seed = 5, 12345
    print("case: cv_grouped scaled n=30000 p=60 K=5", flush=True)
    pr = workloads.cv_grouped(n=30_000, p=60, group_size=10, active_groups=2, seed_tag=215)
    pens = ["grp_lasso", "lasso", dict(kind="mcp", gamma=3.0)]
    res = oem.cv(_cuda(pr.X), _cuda(pr.y), K, seed, pens, nlambda=20, tol=TOL, groups=pr.groups)
    torch.cuda.synchronize()
    ref = oracle.cv(pr.X, pr.y, K, seed, pens, groups=pr.groups, nlambda=20, tol=TOL)
    _assert_paths(res["beta"].cpu().numpy(), ref["full"]["beta"], what="cv full")
    bf = res["beta_folds"].cpu().numpy()
    for k in range(K):
        _assert_paths(bf[k], ref["folds"][k]["beta"], what=f"cv fold {k}")
    cvm = res["cvm"].cpu().numpy()
    assert np.allclose(cvm, ref["cvm"], rtol=1e-9, atol=0)
    assert np.allclose(res["cvsd"].cpu().numpy(), ref["cvsd"], rtol=1e-6, atol=1e-14)
    im = res["i_min"].cpu().numpy()
    for q in range(3):
        # either index is correct when the two curve values agree to 1e-9
        a, b = im[q], ref["i_min"][q]
        assert a == b or abs(ref["cvm"][q, a] - ref["cvm"][q, b]) <= 1e-9 * ref["cvm"][q, b]
    assert res["best"].item() == ref["best"] or abs(
        ref["cvm"][res["best"].item()].min() - ref["cvm"][ref["best"]].min()) <= 1e-9
    # lambda_1se: the first index whose cvm is within one standard error of
    # the minimum; the GPU's index must satisfy the oracle's rule, and any
    # index before it must not (ties within 1e-9 accepted either way)
    i1 = res["i_1se"].cpu().numpy()
    for q in range(3):
        a, b = int(i1[q]), int(ref["i_1se"][q])
        thr = ref["cvm"][q, ref["i_min"][q]] + ref["cvsd"][q, ref["i_min"][q]]
        assert a == b or abs(ref["cvm"][q, a] - thr) <= 1e-9 * thr or abs(
            ref["cvm"][q, b] - thr) <= 1e-9 * thr, (q, a, b)
        assert ref["cvm"][q, a] <= thr * (1 + 1e-9)


def test_cv_parity_grouped_large_p():
    """CV with p = 200 (streaming kernel for every fold): K=3, three penalties."""
    oem = _oem()
    K, seed = 3, 777
    print("case: cv_grouped scaled n=12000 p=200 K=3", flush=True)
    pr = workloads.cv_grouped(n=12_000, p=200, group_size=10, active_groups=3, seed_tag=218)
    pens = ["grp_lasso", "lasso", dict(kind="mcp", gamma=3.0)]
    res = oem.cv(_cuda(pr.X), _cuda(pr.y), K, seed, pens, nlambda=12, tol=TOL, groups=pr.groups)
    torch.cuda.synchronize()
    ref = oracle.cv(pr.X, pr.y, K, seed, pens, groups=pr.groups, nlambda=12, tol=TOL)
    _assert_paths(res["beta"].cpu().numpy(), ref["full"]["beta"], what="cv full p=200")
    bf = res["beta_folds"].cpu().numpy()
    for k in range(K):
        _assert_paths(bf[k], ref["folds"][k]["beta"], what=f"cv fold {k} p=200")
    assert np.allclose(res["cvm"].cpu().numpy(), ref["cvm"], rtol=1e-9, atol=0)


def test_cv_equals_naive_refits():
    """oem_cv on fold statistics == separate fits on the physically split rows."""
    oem = _oem()
    K, seed = 4, 99
    pr = workloads.tall_multi(n=12_000, p=16, seed_tag=216)
    res = oem.cv(_cuda(pr.X), _cuda(pr.y), K, seed, ["lasso"], nlambda=15, tol=TOL)
    lam = res["lambda_"].cpu().numpy()
    f = oracle.fold_ids(seed, pr.X.shape[0], K)
    for k in range(K):
        Xt = np.ascontiguousarray(pr.X[f != k])
        r = oem.fit(_cuda(Xt), _cuda(pr.y[f != k]), ["lasso"], nlambda=15, lambdas=lam, tol=TOL)
        _assert_paths(res["beta_folds"].cpu().numpy()[k], r["beta"].cpu().numpy(), tol=1e-9,
                      what=f"naive fold {k}")


@pytest.mark.parametrize("p,rho,corr", [(1, 0.0, "ar1"), (5, 0.3, "ar1"), (64, -0.6, "ar1"),
                                        (100, 0.5, "ar1"), (128, 0.25, "cs"), (129, -0.4, "ar1"),
                                        (300, 0.3, "ar1"), (520, 0.3, "ar1"), (1100, 0.2, "cs")])
def test_d_matches_jacobi(p, rho, corr):
    """d = lambda_1(Gs)(1 + 1e-10) from Lanczos agrees with the oracle's Jacobi."""
    oem = _oem()
    n = 4000 + 20 * p if p <= 600 else 3 * p
    print(f"case: d p={p} rho={rho} {corr}", flush=True)
    X = workloads.draw_rows(n, p, rho, np.float32, workloads.subseed(300, p), correlation=corr)
    y = workloads.response(X, np.ones(p) / p, 1.0, workloads.subseed(301, p))
    res = oem.fit(_cuda(X), _cuda(y), ["lasso"], nlambda=1)
    G, b, yy, nn = oracle.gram_train(X, y, -1)
    st = oracle.prepare(G, b, yy, nn)
    d_ref = oracle.oem_d(st["Gs"])
    assert abs(res["d"].item() - d_ref) <= 1e-12 * d_ref


@pytest.mark.parametrize("precision", ["split_bf16"])
@pytest.mark.parametrize("n,p", [(200_000, 100), (400_000, 300)])
def test_mixed_gram_paths_within_1e6(precision, n, p):
    """Paths on the split-BF16 Gram match the FP64 paths to 1e-6 relative.

    Error model: each split-BF16 product drops terms of relative size about
    2^-18, random in sign, so the Gram error relative to ||G|| is about
    2^-18 sqrt(p / n) and the coefficient error that times the condition
    number; the tall shapes here (n / p >= 1000) keep it well below 1e-6.
    The FP64 reference runs the oracle's path pipeline on the FP64 Gram
    formed by a library matrix product (the oracle's own row loops would take
    minutes at this size)."""
    oem = _oem()
    print(f"case: mixed gram paths {precision} n={n} p={p}", flush=True)
    pr = workloads.tall_multi(n=n, p=p, seed_tag=220)
    pens = [dict(kind="lasso"), dict(kind="enet", alpha=0.5), dict(kind="mcp", gamma=3.0),
            dict(kind="scad", gamma=3.7)]
    X64 = pr.X.astype(np.float64)
    st = oracle.prepare(X64.T @ X64, X64.T @ pr.y, float(pr.y @ pr.y), n)
    lam = oracle.lambda_sequences(st["cs"], pens, 30, 1e-3)
    ref = oracle.fit_from_stats(st, pens, lam, tol=TOL)
    res = oem.fit(_cuda(pr.X), _cuda(pr.y), pens, precision=precision, nlambda=30, tol=TOL,
                  lambdas=lam)
    b = res["beta"].cpu().numpy()
    worst = 0.0
    for q in range(4):
        for l in range(1, 30):
            r = ref["beta"][q, l]
            worst = max(worst, np.abs(b[q, l] - r).max() / np.abs(r).max())
    print(f"  worst coefficient error {worst:.3e}")
    assert worst <= 1e-6
