"""Pins of the oracle's cross-validation pieces (Section 3, Section 5.5 outputs)."""
import numpy as np
import pytest

import oracle
from oracle import Penalty
import workloads


def test_heldout_mse_equals_gram_identity():
    """sum_{i in k}(y_i - x_i^T b)^2 = yy_k - 2 b^T b_k + b^T G_k b."""
    pr = workloads.tall_multi(n=6000, p=9, seed_tag=41)
    K, seed = 5, 99
    G, b, yy, nk = oracle.gram_folds(pr.X, pr.y, K, seed)
    rng = np.random.default_rng(0)
    betas = rng.normal(size=(4, 9))
    for k in range(K):
        direct = oracle.heldout_mse(pr.X, pr.y, k, K, seed, betas)
        gram = (yy[k] - 2 * betas @ b[k] + np.einsum("li,ij,lj->l", betas, G[k], betas)) / nk[k]
        assert np.max(np.abs(direct - gram) / direct) <= 1e-12


def test_selection_rules_on_hand_made_curves():
    # two penalties, 3 folds of equal size, 5 lambdas
    mse = np.array([
        [[5, 4, 3, 3.2, 3.5], [5, 4, 3, 3.2, 3.5], [5, 4.2, 3.6, 3.2, 3.5]],
        [[5, 4, 2.9, 3, 3], [5, 4, 3.1, 3, 3], [5, 4, 3.0, 3, 3]],
    ], dtype=float)
    nk = np.array([10, 10, 10])
    s = oracle.select(mse, nk)
    cvm0 = mse[0].mean(axis=0)
    assert np.allclose(s["cvm"][0], cvm0)
    sd0 = np.sqrt(((mse[0] - cvm0) ** 2).sum(axis=0) / (30 * 2) * 10)
    assert np.allclose(s["cvsd"][0], sd0)
    assert s["i_min"][0] == int(np.argmin(cvm0))
    thr = cvm0[s["i_min"][0]] + sd0[s["i_min"][0]]
    assert s["i_1se"][0] == int(np.nonzero(cvm0 <= thr)[0][0])
    assert s["i_min"][1] == 2          # tie between l=2,3,4 (all 3.0) -> first
    assert s["best"] == 1


def test_fast_cv_equals_naive_refits():
    """Training statistics from the fold partition equal a refit on the split rows."""
    pr = workloads.tall_multi(n=3000, p=8, seed_tag=42)
    K, seed = 4, 5
    pens = [Penalty("lasso"), Penalty("mcp", gamma=3.0)]
    r = oracle.cv(pr.X, pr.y, K, seed, pens, nlambda=10)
    f = oracle.fold_ids(seed, 3000, K)
    for k in range(K):
        Xt = np.ascontiguousarray(pr.X[f != k])
        yt = pr.y[f != k]
        naive = oracle.fit(Xt, yt, pens, lambdas=r["full"]["lambda"])
        assert np.max(np.abs(naive["beta"] - r["folds"][k]["beta"])) <= 1e-12 * np.abs(
            naive["beta"]).max()
        Xh = pr.X[f == k].astype(np.float64)
        for q in range(2):
            res = ((pr.y[f == k][None, :] - naive["beta"][q] @ Xh.T) ** 2).mean(axis=1)
            assert np.allclose(res, r["mse"][q, k], rtol=1e-12)
    assert r["nk"].sum() == 3000
    assert 0 <= r["best"] < 2
