"""GPU parity of penalised logistic regression (oem_logistic_path, Section 4:
proximal Newton with an OEM inner loop) against the oracle, through the C
ABI.

Tolerance: both sides run the same nested iteration (Newton steps, inner
OEM updates to tol, Newton stopping rule) from the same warm starts, with
the inner and Newton tolerances at 1e-12; the weighted statistics differ
only by rounding (sum order, exp), so the coefficients agree to about the
stopping tolerances amplified by the conditioning: 1e-9 relative to each
solution's largest coefficient, with equal active sets."""
import numpy as np
import pytest

import oracle
import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-9


def _oem():
    import paper_1801_09661_amd as oem
    return oem


def _cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _compare(got, ref, tol=TOL, what=""):
    for q in range(ref.shape[0]):
        for l in range(ref.shape[1]):
            s = np.abs(ref[q, l]).max()
            if s == 0.0:
                assert np.all(got[q, l] == 0.0), (what, q, l)
                continue
            err = np.abs(got[q, l] - ref[q, l]).max() / s
            assert err <= tol, f"{what} pen {q} lambda {l}: rel err {err:.2e}"
            assert np.array_equal(got[q, l] != 0, ref[q, l] != 0), (what, q, l)


@pytest.mark.parametrize("p,n,bound", [(12, 20_000, False), (70, 8_000, False), (150, 3_000, False),
                                       (40, 12_000, True)])
def test_logistic_parity(p, n, bound):
    oem = _oem()
    print(f"case: logistic p={p} n={n} hessian_bound={bound}", flush=True)
    pr = workloads.logistic(n=n, p=p, seed_tag=800 + p)
    groups = (np.arange(p) // 4).astype(np.int32)
    pens = ["lasso", dict(kind="mcp", gamma=3.0), "grp_lasso"]
    kw = dict(nlambda=12, lambda_min_ratio=0.02, tol=1e-12, newton_tol=1e-12,
              newton_maxit=5000 if bound else 100)
    ref = oracle.logistic_path(pr.X, pr.y, pens, groups=groups, hessian_bound=bound, **kw)
    res = oem.logistic_path(_cuda(pr.X), _cuda(pr.y), pens, groups=groups, hessian_bound=bound, **kw)
    torch.cuda.synchronize()
    assert res["status"] == oem.OEM_OK and ref["status"] == 0
    assert np.allclose(res["lambda_"].cpu().numpy(), ref["lambda_"], rtol=1e-12, atol=0)
    _compare(res["beta"].cpu().numpy(), ref["beta"], what=f"p={p}")
    assert np.all(res["kkt"].cpu().numpy() <= 1e-8)
    assert np.allclose(res["obj"].cpu().numpy(), ref["obj"], rtol=1e-10, atol=0)
    nt = res["newton"].cpu().numpy()
    assert np.all(nt > 0)
    if not bound:
        assert np.all(np.abs(nt - ref["newton"]) <= 1)


def test_logistic_fp64_x_explicit_lambda_and_errors():
    oem = _oem()
    print("case: logistic FP64 X, explicit lambda, errors", flush=True)
    pr = workloads.logistic(n=15_000, p=20, seed_tag=820, dtype=np.float64)
    lam = np.geomspace(0.05, 0.002, 8)[None, :]
    ref = oracle.logistic_path(pr.X, pr.y, ["lasso"], lambdas=lam, tol=1e-12, newton_tol=1e-12)
    res = oem.logistic_path(_cuda(pr.X), _cuda(pr.y), ["lasso"], nlambda=8, lambdas=lam, tol=1e-12,
                            newton_tol=1e-12)
    torch.cuda.synchronize()
    _compare(res["beta"].cpu().numpy(), ref["beta"], what="fp64 X")
    X, y = _cuda(pr.X), _cuda(pr.y)
    with pytest.raises(oem.OemError) as e:
        oem.logistic_path(X, y, ["lasso"], nlambda=3, newton_tol=0.0)
    assert e.value.code == oem.OEM_E_INVAL
    big = torch.zeros((4, 2049), dtype=torch.float32, device="cuda")
    with pytest.raises(oem.OemError) as e:
        oem.logistic_path(big, torch.zeros(4, dtype=torch.float64, device="cuda"), ["lasso"], nlambda=3)
    assert e.value.code == oem.OEM_E_INVAL
