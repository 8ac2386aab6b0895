"""Pins of the oracle's intercept option (centred columns and response, an
unpenalised intercept beta0 = ybar - xbar^T beta; the glmnet-style option the
model of Section 2.1 leaves out) and of the held-out error with an intercept.

* shifting y by a constant moves only beta0; shifting column j moves beta0
  by -shift * beta_j and leaves beta alone;
* the intercept model equals the lasso on [X, 1] with the constant column
  unpenalised (weight 0), solved by the same OEM code without centring;
* at lambda_max beta = 0 and beta0 = mean(y); with lambda = 0 the fit is
  least squares with an intercept (numpy lstsq on [1, X]);
* the CV error identity with an intercept: the held-out residual sum of
  squares equals yy_k - 2 b0 sum y - 2 beta^T b_k + n_k b0^2 + 2 b0 beta^T
  colsum_k + beta^T G_k beta, from the fold sums.
"""
import numpy as np
import pytest

import oracle
from oracle import Penalty
import workloads


def _data(n=4000, p=12, seed_tag=80, shift=True):
    pr = workloads.tall_multi(n=n, p=p, seed_tag=seed_tag)
    X = pr.X.astype(np.float64)
    y = pr.y.copy()
    if shift:
        rng = np.random.default_rng(seed_tag)
        X = X + rng.uniform(-2.0, 2.0, size=p)[None, :]
        y = y + 5.0
    return np.ascontiguousarray(X), y


PENS = ["lasso", dict(kind="mcp", gamma=3.0), dict(kind="enet", alpha=0.5)]


def test_response_and_column_shifts():
    X, y = _data()
    a = oracle.fit(X, y, PENS, nlambda=15, lambda_min_ratio=1e-2, intercept=True)
    b = oracle.fit(X, y + 3.25, PENS, nlambda=15, lambda_min_ratio=1e-2, intercept=True)
    assert np.allclose(a["lambda"], b["lambda"], rtol=1e-12, atol=0)
    assert np.allclose(b["beta"], a["beta"], rtol=0, atol=1e-11 * np.abs(a["beta"]).max())
    assert np.allclose(b["beta0"], a["beta0"] + 3.25, rtol=0, atol=1e-10)
    Xs = X.copy()
    Xs[:, 4] += 7.5
    c = oracle.fit(Xs, y, PENS, nlambda=15, lambda_min_ratio=1e-2, intercept=True)
    assert np.allclose(c["beta"], a["beta"], rtol=0, atol=1e-10 * np.abs(a["beta"]).max())
    assert np.allclose(c["beta0"], a["beta0"] - 7.5 * a["beta"][:, :, 4], rtol=0, atol=1e-9)


def test_equals_unpenalised_constant_column():
    """No standardisation on either side: the centred lasso and the lasso on
    [X, 1] with weight 0 on the constant column have the same minimiser."""
    X, y = _data(n=3000, p=8, seed_tag=81)
    n, p = X.shape
    a = oracle.fit(X, y, ["lasso"], nlambda=10, lambda_min_ratio=0.05, standardize=False,
                   intercept=True, tol=1e-13)
    Xa = np.ascontiguousarray(np.hstack([X, np.ones((n, 1))]))
    w = np.r_[np.ones(p), 0.0]
    b = oracle.fit(Xa, y, ["lasso"], w=w, lambdas=a["lambda"], standardize=False, tol=1e-13,
                   maxit=2_000_000)
    for l in range(10):
        s = max(np.abs(a["beta"][0, l]).max(), 1.0)
        assert np.abs(b["beta"][0, l, :p] - a["beta"][0, l]).max() <= 1e-8 * s
        assert abs(b["beta"][0, l, p] - a["beta0"][0, l]) <= 1e-8 * max(1.0, abs(a["beta0"][0, l]))


def test_lambda_max_and_least_squares_ends():
    X, y = _data(n=2500, p=6, seed_tag=82)
    a = oracle.fit(X, y, ["lasso"], nlambda=5, lambda_min_ratio=0.1, intercept=True)
    assert np.all(a["beta"][0, 0] == 0.0)
    assert a["beta0"][0, 0] == pytest.approx(float(np.mean(y)), rel=1e-14)
    ols = oracle.fit(X, y, ["lasso"], lambdas=np.array([[0.0]]), intercept=True, tol=1e-14,
                     maxit=5_000_000)
    A = np.hstack([np.ones((X.shape[0], 1)), X])
    coef = np.linalg.lstsq(A, y, rcond=None)[0]
    assert abs(ols["beta0"][0, 0] - coef[0]) <= 1e-8 * max(1.0, abs(coef[0]))
    assert np.abs(ols["beta"][0, 0] - coef[1:]).max() <= 1e-8 * np.abs(coef[1:]).max()


def test_cv_error_identity_with_intercept():
    """Held-out residuals from rows (the oracle's CV) against the Gram-form
    expression written out here from the held-out fold's sums."""
    X, y = _data(n=6000, p=10, seed_tag=83)
    K, seed = 4, 7
    res = oracle.cv(X, y, K, seed, ["lasso"], nlambda=8, lambda_min_ratio=0.05, intercept=True)
    fid = oracle.fold_ids(seed, X.shape[0], K)
    for k in range(K):
        m = fid == k
        Xk, yk = X[m], y[m]
        G, bk, yy, nk = Xk.T @ Xk, Xk.T @ yk, yk @ yk, m.sum()
        cs, ys = Xk.sum(0), yk.sum()
        beta, b0 = res["folds"][k]["beta"][0], res["folds"][k]["beta0"][0]
        for l in range(8):
            bt = beta[l]
            sse = (yy - 2 * b0[l] * ys - 2 * bt @ bk + nk * b0[l] ** 2 + 2 * b0[l] * bt @ cs
                   + bt @ G @ bt)
            assert sse / nk == pytest.approx(res["mse"][0, k, l], rel=1e-9)
