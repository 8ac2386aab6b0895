"""GPU parity of group MCP, group SCAD and the sparse group lasso (Section 2.2,
eqs. gmcp, gscad, sglasso) against the oracle, FP64 form, through the C ABI.

Tolerance as for the other penalties: same d, same lambda, same stopping
rule, so per (penalty, lambda) max|beta_gpu - beta_oracle| <= 1e-10 *
max|beta_oracle| and equal active sets.
"""
import numpy as np
import pytest

import oracle
import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-10
PENS = [dict(kind="grp_mcp", gamma=3.0), dict(kind="grp_scad", gamma=3.7),
        dict(kind="sgl", tau=0.3)]


def _oem():
    import paper_1801_09661_amd as oem
    return oem


def _cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _assert_paths(b_gpu, b_or, tol=TOL, what=""):
    for q in range(b_or.shape[0]):
        for l in range(b_or.shape[1]):
            ref, got = b_or[q, l], b_gpu[q, l]
            scale = np.abs(ref).max()
            if scale == 0.0:
                assert np.all(got == 0.0), f"{what} pen {q} lambda {l}: expected all-zero"
                continue
            err = np.abs(got - ref).max() / scale
            assert err <= tol, f"{what} pen {q} lambda {l}: rel err {err:.3e}"
            assert np.array_equal(got != 0, ref != 0), f"{what} pen {q} lambda {l}: active set"


@pytest.mark.parametrize("p,gs,n", [(20, 4, 12_000), (63, 5, 20_000), (130, 10, 20_000),
                                    (301, 7, 15_000)])
def test_group_penalties_parity(p, gs, n):
    """Contiguous groups with a ragged last group (p mod size != 0), p spanning
    one to several 64-lane tiles; the lambda grid is the GPU's own and must
    match the oracle's."""
    oem = _oem()
    print(f"case: group penalties p={p} group size {gs} n={n}", flush=True)
    pr = workloads.cv_grouped(n=n, p=p, group_size=gs, active_groups=3, seed_tag=300 + p)
    res = oem.fit(_cuda(pr.X), _cuda(pr.y), PENS, nlambda=25, lambda_min_ratio=1e-2, tol=TOL,
                  groups=pr.groups)
    torch.cuda.synchronize()
    ref = oracle.fit(pr.X, pr.y, PENS, groups=pr.groups, nlambda=25, lambda_min_ratio=1e-2, tol=TOL)
    assert abs(res["d"].item() - ref["d"]) <= 1e-12 * ref["d"]
    assert np.allclose(res["lambda_"].cpu().numpy(), ref["lambda"], rtol=1e-13, atol=0)
    _assert_paths(res["beta"].cpu().numpy(), ref["beta"], what=f"p={p}")
    assert np.all(res["kkt"].cpu().numpy() <= 1e-8)
    assert np.allclose(res["obj"].cpu().numpy(), ref["obj"], rtol=1e-12, atol=0)
    it = res["iters"].cpu().numpy()
    assert np.all(it > 0) and np.all(np.abs(it - ref["iters"]) <= 1)


def test_shuffled_groups_weights_and_tau_range():
    """Non-contiguous groups, variable and group weights, and the sparse group
    lasso at tau in {0, 0.7, 1} (0 is the group lasso, 1 the lasso)."""
    oem = _oem()
    print("case: shuffled groups, weights, tau sweep p=48", flush=True)
    pr = workloads.cv_grouped(n=15_000, p=48, group_size=6, active_groups=3, seed_tag=320)
    rng = np.random.default_rng(321)
    groups = rng.permutation(pr.groups).astype(np.int32)
    w = rng.uniform(0.5, 2.0, size=48)
    cg = rng.uniform(1.0, 3.0, size=int(groups.max()) + 1)
    pens = [dict(kind="sgl", tau=0.0), dict(kind="sgl", tau=0.7), dict(kind="sgl", tau=1.0),
            dict(kind="grp_mcp", gamma=2.5), dict(kind="grp_scad", gamma=4.0)]
    res = oem.fit(_cuda(pr.X), _cuda(pr.y), pens, nlambda=20, lambda_min_ratio=1e-2, tol=TOL,
                  groups=groups, w=w, cg=cg)
    torch.cuda.synchronize()
    ref = oracle.fit(pr.X, pr.y, pens, groups=groups, w=w, cg=cg, nlambda=20,
                     lambda_min_ratio=1e-2, tol=TOL)
    assert np.allclose(res["lambda_"].cpu().numpy(), ref["lambda"], rtol=1e-13, atol=0)
    _assert_paths(res["beta"].cpu().numpy(), ref["beta"], what="shuffled")
    assert np.all(res["kkt"].cpu().numpy() <= 1e-8)


def test_group_penalties_cv_parity():
    """K = 4 hashed folds: every fold's path, the CV curve and the selection
    against the oracle's refits on physically split rows."""
    oem = _oem()
    K, seed = 4, 97
    print("case: group penalties CV K=4 p=40", flush=True)
    pr = workloads.cv_grouped(n=16_000, p=40, group_size=5, active_groups=3, seed_tag=330)
    res = oem.cv(_cuda(pr.X), _cuda(pr.y), K, seed, PENS, nlambda=20, lambda_min_ratio=1e-2,
                 tol=TOL, groups=pr.groups)
    torch.cuda.synchronize()
    ref = oracle.cv(pr.X, pr.y, K, seed, PENS, groups=pr.groups, nlambda=20, lambda_min_ratio=1e-2,
                    tol=TOL)
    _assert_paths(res["beta"].cpu().numpy(), ref["full"]["beta"], what="full")
    bf = res["beta_folds"].cpu().numpy()
    for k in range(K):
        _assert_paths(bf[k], ref["folds"][k]["beta"], what=f"fold {k}")
    assert np.allclose(res["cvm"].cpu().numpy(), ref["cvm"], rtol=1e-9, atol=0)
    assert np.allclose(res["cvsd"].cpu().numpy(), ref["cvsd"], rtol=1e-7, atol=1e-15)
    assert np.array_equal(res["i_min"].cpu().numpy(), ref["i_min"])
    assert np.array_equal(res["i_1se"].cpu().numpy(), ref["i_1se"])
    assert int(res["best"].item()) == ref["best"]


def test_group_penalty_argument_errors():
    oem = _oem()
    print("case: group penalty argument errors", flush=True)
    pr = workloads.cv_grouped(n=2000, p=10, group_size=5, active_groups=1, seed_tag=340)
    X, y = _cuda(pr.X), _cuda(pr.y)
    for pens, groups, what in [([dict(kind="sgl", tau=1.5)], pr.groups, "tau"),
                               ([dict(kind="sgl", tau=-0.1)], pr.groups, "tau"),
                               ([dict(kind="grp_mcp", gamma=3.0)], None, "groups"),
                               ([dict(kind="grp_scad", gamma=1.5)], pr.groups, "gamma")]:
        with pytest.raises(oem.OemError) as e:
            oem.fit(X, y, pens, nlambda=5, groups=groups)
        assert e.value.code == oem.OEM_E_INVAL, what
    # tau belongs to the sparse group lasso only
    with pytest.raises(oem.OemError) as e:
        oem.fit(X, y, [oem.Penalty("lasso", tau=0.2)], nlambda=5)
    assert e.value.code == oem.OEM_E_INVAL
