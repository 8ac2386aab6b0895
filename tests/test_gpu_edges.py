"""GPU parity on the cases the main parity files leave out: paths with
p > 1000 (streaming kernel) against the oracle, FP64 X with folds, the
mixed form's active-set rule, small p in the Gram pass, and the error
statuses of the boundary (non-finite statistics, a fold with no held-out
rows)."""
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


def _assert_paths(b_gpu, b_or, tol=TOL, what="", first_is_knife_edge=False):
    """Element-wise parity of (penalty, lambda, p) paths at `tol` relative to
    each solution's largest coefficient, and equal active sets.  With
    first_is_knife_edge the first lambda is lambda_max of a Gram rounded
    differently from the GPU's: there the GPU may keep a coordinate whose
    |c_j| exceeds lambda by a rounding error, so its coefficients are only
    required to be at rounding level of the next solution."""
    for q in range(b_or.shape[0]):
        for l in range(b_or.shape[1]):
            ref, got = b_or[q, l], b_gpu[q, l]
            scale = np.abs(ref).max()
            if l == 0 and first_is_knife_edge:
                nxt = np.abs(b_or[q, 1]).max() if b_or.shape[1] > 1 else 1.0
                assert np.abs(got).max() <= 1e-10 * nxt, f"{what} pen {q} lambda 0"
                continue
            if scale == 0.0:
                assert np.all(got == 0.0), f"{what} pen {q} lambda {l}"
                continue
            err = np.abs(got - ref).max() / scale
            assert err <= tol, f"{what} pen {q} lambda {l}: rel err {err:.3e}"
            assert np.array_equal(got != 0, ref != 0), f"{what} pen {q} lambda {l}: active set"


@pytest.mark.parametrize("p,n,pens", [
    (1100, 8000, ["lasso", dict(kind="mcp", gamma=3.0)]),
    (1942, 12000, ["lasso"]),
])
def test_paths_parity_large_p(p, n, pens):
    """p in (1000, 2048], active sets growing past a thousand coordinates
    (working-set kernels, then the streaming kernel).  The reference is the
    oracle's path pipeline on the FP64 Gram of a library product, with d from
    a library symmetric eigen-solver (the oracle's Jacobi, pinned against the
    same solver, would take minutes at this size)."""
    oem = _oem()
    print(f"case: large-p paths p={p} n={n}", flush=True)
    pr = workloads.tall_multi(n=n, p=p, seed_tag=250 + p % 97)
    X64 = pr.X.astype(np.float64)
    st = oracle.prepare(X64.T @ X64, X64.T @ pr.y, float(pr.y @ pr.y), n)
    d_ref = float(np.linalg.eigvalsh(st["Gs"]).max()) * (1 + 1e-10)
    lam = oracle.lambda_sequences(st["cs"], pens, 12, 1e-3)
    res = oem.fit(_cuda(pr.X), _cuda(pr.y), pens, nlambda=12, lambdas=lam, tol=TOL)
    torch.cuda.synchronize()
    assert abs(res["d"].item() - d_ref) <= 1e-12 * d_ref
    ref = oracle.fit_from_stats(st, pens, lam, tol=TOL, d=d_ref)
    b = res["beta"].cpu().numpy()
    _assert_paths(b, ref["beta"], what=f"p={p}", first_is_knife_edge=True)
    assert (ref["beta"][0, -1] != 0).sum() > 128       # the streaming kernel ran
    assert np.all(res["kkt"].cpu().numpy() <= 1e-8)


def test_group_lasso_parity_large_p_streaming():
    """Group lasso at p = 1100 with 16 active groups of 10: the path moves from
    the two-wave and four-wave working sets (at most 12 groups of 10) to the
    streaming kernel.  Reference as in the large-p test above: the oracle's
    path pipeline on a library FP64 Gram, d from a library eigen-solver."""
    oem = _oem()
    print("case: group lasso p=1100 n=6000, 16 active groups", flush=True)
    pr = workloads.cv_grouped(n=6000, p=1100, group_size=10, active_groups=16, seed_tag=251)
    X64 = pr.X.astype(np.float64)
    st = oracle.prepare(X64.T @ X64, X64.T @ pr.y, float(pr.y @ pr.y), 6000)
    d_ref = float(np.linalg.eigvalsh(st["Gs"]).max()) * (1 + 1e-10)
    pens = ["grp_lasso"]
    lam = oracle.lambda_sequences(st["cs"], pens, 15, 2e-2, groups=pr.groups)
    res = oem.fit(_cuda(pr.X), _cuda(pr.y), pens, nlambda=15, lambdas=lam, tol=TOL, groups=pr.groups)
    torch.cuda.synchronize()
    assert abs(res["d"].item() - d_ref) <= 1e-12 * d_ref
    ref = oracle.fit_from_stats(st, pens, lam, groups=pr.groups, tol=TOL, d=d_ref)
    _assert_paths(res["beta"].cpu().numpy(), ref["beta"], what="grp p=1100", first_is_knife_edge=True)
    assert (ref["beta"][0, -1] != 0).sum() > 120       # more than 12 groups: the streaming kernel ran
    assert np.all(res["kkt"].cpu().numpy() <= 1e-8)


def test_fp64_x_with_folds():
    """FP64 X and K = 3 hashed folds: CV parity against the oracle."""
    oem = _oem()
    K, seed = 3, 4242
    print("case: FP64 X, K=3 CV", flush=True)
    pr = workloads.small_lasso(n=9000, p=24, seed_tag=260)
    assert pr.X.dtype == np.float64
    pens = ["lasso", dict(kind="scad", gamma=3.7)]
    res = oem.cv(_cuda(pr.X), _cuda(pr.y), K, seed, pens, nlambda=15, tol=TOL)
    torch.cuda.synchronize()
    ref = oracle.cv(pr.X, pr.y, K, seed, pens, nlambda=15, tol=TOL)
    _assert_paths(res["beta"].cpu().numpy(), ref["full"]["beta"], what="fp64 X full")
    bf = res["beta_folds"].cpu().numpy()
    for k in range(K):
        _assert_paths(bf[k], ref["folds"][k]["beta"], what=f"fp64 X fold {k}")
    assert np.allclose(res["cvm"].cpu().numpy(), ref["cvm"], rtol=1e-9, atol=0)
    with oem.Gram(24, K, "fp64", torch.float64, seed) as g:
        g.add(_cuda(pr.X), _cuda(pr.y))
        nk = g.export()[3].cpu().numpy()
    assert np.array_equal(nk, np.bincount(oracle.fold_ids(seed, 9000, K), minlength=K))


def test_mixed_active_set_rule():
    """Split-BF16 Gram: active sets equal the FP64 oracle's except at
    coordinates whose stationarity margin | |g_j| - lambda | / lambda is
    below 1e-5 (undecidable at 1e-6 accuracy); those must be tiny."""
    oem = _oem()
    print("case: mixed active-set rule n=200000 p=100", flush=True)
    pr = workloads.tall_multi(n=200_000, p=100, seed_tag=261)
    pens = [dict(kind="lasso"), dict(kind="mcp", gamma=3.0)]
    X64 = pr.X.astype(np.float64)
    st = oracle.prepare(X64.T @ X64, X64.T @ pr.y, float(pr.y @ pr.y), pr.X.shape[0])
    lam = oracle.lambda_sequences(st["cs"], pens, 40, 1e-3)
    ref = oracle.fit_from_stats(st, pens, lam, tol=TOL)
    res = oem.fit(_cuda(pr.X), _cuda(pr.y), pens, precision="split_bf16", nlambda=40,
                  lambdas=lam, tol=TOL)
    bm = res["beta"].cpu().numpy() * st["s"][None, None, :]      # standardised scale
    mism = 0
    for q in range(2):
        for l in range(1, 40):
            br = ref["beta_std"][q, l]
            g = st["Gs"] @ br - st["cs"]
            margin = np.abs(np.abs(g) - lam[q, l]) / lam[q, l]
            diff = (bm[q, l] != 0) != (br != 0)
            mism += int(diff.sum())
            assert np.all(margin[diff] < 1e-5), (q, l)
            assert np.all(np.abs(bm[q, l][diff]) <= 1e-6 * np.abs(br).max()), (q, l)
            assert np.abs(bm[q, l] - br).max() <= 1e-6 * np.abs(br).max()
    print(f"  active-set mismatches (all within the margin rule): {mism}")


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5])
@pytest.mark.parametrize("precision", ["fp64", "split_bf16", "bf16"])
def test_gram_small_p_integer_exact(p, precision):
    """Integer X (exact in every form) with p at or below one 16-byte load;
    the tensor's storage ends with the last row."""
    oem = _oem()
    n = 3001
    X = workloads.integer_rows(n, p, seed_tag=262 + p).astype(np.float32)
    y = workloads.integer_response(n, seed_tag=263 + p)
    Xd = torch.from_numpy(X).cuda()
    with oem.Gram(p, 1, precision, torch.float32) as g:
        g.add(Xd, _cuda(y))
        G, b, yy, nk = (t.cpu().numpy() for t in g.export())
    Gr, br, yyr, nkr = oracle.gram_folds(X, y)
    assert np.array_equal(G, Gr) and np.array_equal(b, br)
    assert yy[0] == yyr[0] and nk[0] == nkr[0] == n


def test_nonfinite_statistics_rejected():
    """An imported Gram with a NaN entry gives a clear error status, not NaN
    coefficients with OEM_OK."""
    oem = _oem()
    print("case: imported Gram with a NaN entry", flush=True)
    p = 6
    rng = np.random.default_rng(3)
    A = rng.normal(size=(50, p))
    G = A.T @ A
    G[2, 3] = G[3, 2] = np.nan
    with oem.Gram(p, 1, "fp64") as g:
        oem.oem_gram_import(g.h, 0, _cuda(G), _cuda(A.T @ rng.normal(size=50)), 1.0, 50)
        with pytest.raises(oem.OemError) as ei:
            g.fit_path(["lasso"], nlambda=4)
        assert ei.value.code == oem.OEM_E_INVAL
        assert "finite" in str(ei.value)
    # an all-zero design: d = 0, rejected the same way
    with oem.Gram(p, 1, "fp64") as g:
        oem.oem_gram_import(g.h, 0, _cuda(np.zeros((p, p))), _cuda(np.zeros(p)), 1.0, 50)
        with pytest.raises(oem.OemError):
            g.fit_path(["lasso"], nlambda=4)


def test_fold_without_heldout_rows_rejected():
    """A fold-id array that leaves fold 2 of 4 empty: the oracle refuses the
    held-out error of that fold, and oem_cv refuses the whole call."""
    oem = _oem()
    print("case: fold with no held-out rows", flush=True)
    pr = workloads.tall_multi(n=4000, p=8, seed_tag=264)
    fid = (np.arange(4000) % 3).astype(np.uint8)
    fid[fid == 2] = 3                                   # ids 0, 1, 3 used; 2 empty
    with pytest.raises(ValueError):
        oracle.heldout_mse(pr.X, pr.y, 2, 4, 0, np.zeros((1, 8)), foldid=fid)
    with oem.Gram(8, 4, "fp64", torch.float32, 0) as g:
        g.add(_cuda(pr.X), _cuda(pr.y), foldid=_cuda(fid))
        with pytest.raises(oem.OemError) as ei:
            g.cv(["lasso"], nlambda=5)
        assert "no held-out rows" in str(ei.value)
