"""Pins of the oracle's penalised logistic regression (Section 4: proximal
Newton with OEM as the inner solver).

* with lambda = 0 the result is the maximum-likelihood estimate, found here
  by plain Newton-Raphson in numpy;
* stationarity of the logistic problem, written out here with numpy, holds
  at every lambda;
* the lasso fixed point equals an independent proximal-gradient (FISTA)
  solve of the same convex problem written here;
* the Hessian-bound variant (w_i = 1/4) reaches the same solution;
* lambda_max is max_j |x~_j^T (y - 1/2)| / n: zero at the first lambda,
  nonzero just below.
"""
import numpy as np
import pytest

import oracle
from oracle import Penalty
import workloads


def _prob(n=4000, p=12, seed_tag=95):
    pr = workloads.logistic(n=n, p=p, seed_tag=seed_tag)
    X = pr.X.astype(np.float64)
    s = np.sqrt((X * X).mean(0))
    return pr, X, s


def _sig(t):
    return 1.0 / (1.0 + np.exp(-t))


def test_unpenalised_is_maximum_likelihood():
    pr, X, s = _prob()
    r = oracle.logistic_path(pr.X, pr.y, ["lasso"], lambdas=np.array([[0.0]]), tol=1e-13,
                             newton_tol=1e-13)
    b = np.zeros(X.shape[1])
    for _ in range(50):
        mu = _sig(X @ b)
        H = X.T @ (X * (mu * (1 - mu))[:, None])
        b = b + np.linalg.solve(H, X.T @ (pr.y - mu))
    assert np.abs(r["beta"][0, 0] - b).max() <= 1e-8 * np.abs(b).max()
    assert r["newton"][0, 0] > 0


def test_stationarity_written_out():
    pr, X, s = _prob(seed_tag=96)
    n = X.shape[0]
    Xs = X / s
    r = oracle.logistic_path(pr.X, pr.y, ["lasso"], nlambda=12, lambda_min_ratio=0.02)
    for l, lam in enumerate(r["lambda_"][0]):
        bt = r["beta"][0, l] * s
        g = -Xs.T @ (pr.y - _sig(Xs @ bt)) / n
        nz = bt != 0
        assert np.all(np.abs(g[~nz]) <= lam * (1 + 1e-9) + 1e-12)
        assert np.all(np.abs(g[nz] + lam * np.sign(bt[nz])) <= 1e-8)
        assert r["kkt"][0, l] <= 1e-8
        loss = np.mean(np.logaddexp(0.0, Xs @ bt) - pr.y * (Xs @ bt))
        assert r["obj"][0, l] == pytest.approx(loss + lam * np.abs(bt).sum(), rel=1e-12)


def test_lasso_equals_fista():
    pr, X, s = _prob(seed_tag=97)
    n = X.shape[0]
    Xs = X / s
    r = oracle.logistic_path(pr.X, pr.y, ["lasso"], nlambda=6, lambda_min_ratio=0.05, tol=1e-13,
                             newton_tol=1e-13)
    Lip = 0.25 * np.linalg.eigvalsh(Xs.T @ Xs / n).max()
    for l, lam in enumerate(r["lambda_"][0]):
        b = np.zeros(X.shape[1]); v = b.copy(); t = 1.0
        for _ in range(20000):
            g = -Xs.T @ (pr.y - _sig(Xs @ v)) / n
            u = v - g / Lip
            bn = np.sign(u) * np.maximum(np.abs(u) - lam / Lip, 0.0)
            tn = (1 + np.sqrt(1 + 4 * t * t)) / 2
            v = bn + (t - 1) / tn * (bn - b)
            if np.abs(bn - b).max() <= 1e-15 * max(np.abs(bn).max(), 1e-300):
                b = bn
                break
            b, t = bn, tn
        got = r["beta"][0, l] * s
        assert np.abs(got - b).max() <= 1e-8 * max(np.abs(b).max(), 1e-12), l


def test_hessian_bound_reaches_the_same_solution():
    pr, X, s = _prob(seed_tag=98)
    kw = dict(nlambda=8, lambda_min_ratio=0.05, tol=1e-13, newton_tol=1e-13)
    a = oracle.logistic_path(pr.X, pr.y, ["lasso", dict(kind="grp_lasso")],
                             groups=np.arange(12) // 3, **kw)
    b = oracle.logistic_path(pr.X, pr.y, ["lasso", dict(kind="grp_lasso")],
                             groups=np.arange(12) // 3, hessian_bound=True, newton_maxit=20000, **kw)
    assert np.all(b["newton"] > 0)
    for q in range(2):
        for l in range(8):
            sc = max(np.abs(a["beta"][q, l]).max(), 1e-12)
            assert np.abs(a["beta"][q, l] - b["beta"][q, l]).max() <= 1e-7 * sc


def test_lambda_max_literal():
    pr, X, s = _prob(seed_tag=99)
    n = X.shape[0]
    want = np.abs((X / s).T @ (pr.y - 0.5)).max() / n
    r = oracle.logistic_path(pr.X, pr.y, ["lasso"], nlambda=5, lambda_min_ratio=0.9)
    assert r["lambda_"][0, 0] == pytest.approx(want, rel=1e-13)
    assert np.all(r["beta"][0, 0] == 0.0)
    r2 = oracle.logistic_path(pr.X, pr.y, ["lasso"], lambdas=np.array([[want * (1 - 1e-6)]]))
    assert np.count_nonzero(r2["beta"][0, 0]) == 1
