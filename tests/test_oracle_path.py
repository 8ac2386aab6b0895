"""Pins of the oracle's OEM path (Section 2.1 iteration, Section 2.2 updates).

Fixed points are checked against closed forms (orthonormal design, lambda = 0
least squares), exhaustive enumeration (lasso, small p), independent
coordinate-descent solvers written here (lasso, elastic net, MCP, SCAD, group
lasso by block descent with a secular-equation solve), stationarity (KKT), and
the majorise-minimise property of each EM step.
"""
import itertools
import math

import numpy as np
import pytest

import oracle
from oracle import Penalty
import workloads


def _stats(X, y, standardize=True):
    G, b, yy, n = oracle.gram_train(X, y, -1)
    return oracle.prepare(G, b, yy, n, standardize)


def _soft(z, t):
    return np.sign(z) * np.maximum(np.abs(z) - t, 0.0)


# ------------------------------------------------------------ orthonormal design

def _hadamard_problem(p=8, n=64, seed=11):
    H = np.array([[1.0]])
    while H.shape[0] < n:
        H = np.block([[H, H], [H, -H]])
    X = np.ascontiguousarray(H[:, 1:p + 1])
    rng = np.random.default_rng(seed)
    y = X @ rng.normal(0, 1.0, size=p) + rng.normal(0, 0.5, size=n)
    return X, y


def _closed_form(kind, c, lam, alpha=0.5, gamma=3.7, groups=None):
    """Textbook thresholding rules for an orthonormal design (d = 1)."""
    if kind == "lasso":
        return _soft(c, lam)
    if kind == "enet":
        return _soft(c, alpha * lam) / (1 + (1 - alpha) * lam)
    if kind == "mcp":   # firm thresholding
        return np.where(np.abs(c) <= gamma * lam, _soft(c, lam) / (1 - 1 / gamma), c)
    if kind == "scad":  # Fan & Li (2001) thresholding rule
        a = gamma
        out = np.where(np.abs(c) <= 2 * lam, _soft(c, lam),
                       np.where(np.abs(c) <= a * lam,
                                ((a - 1) * c - np.sign(c) * a * lam) / (a - 2), c))
        return out
    if kind == "grp_lasso":
        out = np.zeros_like(c)
        for g in np.unique(groups):
            m = groups == g
            nrm = np.linalg.norm(c[m])
            cg = math.sqrt(m.sum())
            out[m] = 0.0 if nrm == 0 else c[m] * max(0.0, 1 - lam * cg / nrm)
        return out
    raise ValueError(kind)


@pytest.mark.parametrize("kind", ["lasso", "enet", "mcp", "scad", "grp_lasso"])
def test_orthonormal_design_gives_thresholding(kind):
    X, y = _hadamard_problem()
    st = _stats(X, y)
    assert np.array_equal(st["Gs"], np.eye(8))
    groups = (np.arange(8) // 2).astype(np.int32) if kind == "grp_lasso" else None
    pen = Penalty(kind, alpha=0.5, gamma=3.7)
    lam = oracle.lambda_grid(oracle.lambda_max(st["cs"], pen, groups), 20, 0.01)
    r = oracle.fit_from_stats(st, [pen], lam[None, :], groups=groups)
    for l in range(20):
        ref = _closed_form(kind, st["cs"], lam[l], groups=groups)
        assert np.max(np.abs(r["beta_std"][0, l] - ref)) <= 1e-9 * max(1.0, np.abs(ref).max())


@pytest.mark.parametrize("kind", ["lasso", "enet", "mcp", "scad", "grp_lasso"])
def test_lambda_max_is_first_all_zero(kind):
    pr = workloads.small_lasso(n=2000, p=10, seed_tag=31)
    st = _stats(pr.X, pr.y)
    groups = (np.arange(10) // 2).astype(np.int32)
    pen = Penalty(kind, alpha=0.5, gamma=3.0)
    lmax = oracle.lambda_max(st["cs"], pen, groups)
    d = oracle.oem_d(st["Gs"])
    lam = np.array([lmax, lmax * (1 - 1e-6)])
    r = oracle.fit_path_std(st["Gs"], st["cs"], st["yyn"], d, pen, lam, groups)
    assert np.all(r["beta_std"][0] == 0.0)
    assert r["iters"][0] == 1
    assert np.any(r["beta_std"][1] != 0.0)


def test_lambda_zero_is_least_squares():
    pr = workloads.tall_multi(n=5000, p=12, seed_tag=32)
    st = _stats(pr.X, pr.y)
    r = oracle.fit_from_stats(st, [Penalty("lasso")], np.zeros((1, 1)), tol=1e-13)
    L = np.linalg.cholesky(st["Gs"])
    ols = np.linalg.solve(L.T, np.linalg.solve(L, st["cs"]))
    assert np.max(np.abs(r["beta_std"][0, 0] - ols)) <= 1e-10 * np.abs(ols).max()
    # and on the original scale against a least-squares solve of the raw data
    raw = np.linalg.lstsq(pr.X.astype(np.float64), pr.y, rcond=None)[0]
    assert np.max(np.abs(r["beta"][0, 0] - raw)) <= 1e-8 * np.abs(raw).max()


# ------------------------------------------------------------ lasso enumeration

def _lasso_enumerate(Gs, cs, lam):
    p = len(cs)
    best = None
    for signs in itertools.product((-1, 0, 1), repeat=p):
        s = np.array(signs, dtype=float)
        A = np.nonzero(s)[0]
        beta = np.zeros(p)
        if len(A):
            beta[A] = np.linalg.solve(Gs[np.ix_(A, A)], cs[A] - lam * s[A])
            if np.any(np.sign(beta[A]) != s[A]):
                continue
        g = Gs @ beta - cs
        I = np.setdiff1d(np.arange(p), A)
        if len(I) and np.any(np.abs(g[I]) > lam * (1 + 1e-12)):
            continue
        best = beta
        break
    return best


def test_lasso_matches_exhaustive_enumeration():
    pr = workloads.tall_multi(n=3000, p=6, seed_tag=33)
    st = _stats(pr.X, pr.y)
    pen = Penalty("lasso")
    lam = oracle.lambda_grid(oracle.lambda_max(st["cs"], pen), 15, 1e-3)
    r = oracle.fit_from_stats(st, [pen], lam[None, :])
    for l in range(1, 15):
        ref = _lasso_enumerate(st["Gs"], st["cs"], lam[l])
        assert ref is not None
        got = r["beta_std"][0, l]
        assert np.max(np.abs(got - ref)) <= 1e-8 * np.abs(ref).max()
        assert np.array_equal(got != 0, ref != 0)


# ------------------------------------------------------------ coordinate descent

def _cd_update(kind, z, lam, alpha, gamma):
    """argmin_b 1/2 b^2 - z b + P(b) (unit curvature), textbook forms."""
    if kind == "lasso":
        return _soft(z, lam)
    if kind == "enet":
        return _soft(z, alpha * lam) / (1 + (1 - alpha) * lam)
    if kind == "mcp":
        return _soft(z, lam) / (1 - 1 / gamma) if abs(z) <= gamma * lam else z
    if kind == "scad":
        if abs(z) <= 2 * lam:
            return _soft(z, lam)
        if abs(z) <= gamma * lam:
            return _soft(z, gamma * lam / (gamma - 1)) / (1 - 1 / (gamma - 1))
        return z
    raise ValueError(kind)


def _coordinate_descent(Gs, cs, lam, kind, alpha=0.5, gamma=3.0, beta0=None):
    p = len(cs)
    beta = np.zeros(p) if beta0 is None else beta0.copy()
    for _ in range(100000):
        mx = 0.0
        for j in range(p):
            z = cs[j] - Gs[j] @ beta + Gs[j, j] * beta[j]
            nb = float(_cd_update(kind, z, lam, alpha, gamma))
            mx = max(mx, abs(nb - beta[j]))
            beta[j] = nb
        if mx <= 1e-15:
            break
    return beta


@pytest.mark.parametrize("kind", ["lasso", "enet", "mcp", "scad"])
def test_matches_coordinate_descent(kind):
    # near-orthogonal design: every objective here is strictly convex, so the
    # stationary point is unique whatever the algorithm.
    pr = workloads.small_lasso(n=4000, p=12, seed_tag=34)
    st = _stats(pr.X, pr.y)
    pen = Penalty(kind, alpha=0.5, gamma=3.7 if kind == "scad" else 3.0)
    lam = oracle.lambda_grid(oracle.lambda_max(st["cs"], pen), 12, 1e-2)
    r = oracle.fit_from_stats(st, [pen], lam[None, :])
    beta = None
    for l in range(12):
        beta = _coordinate_descent(st["Gs"], st["cs"], lam[l], kind, 0.5, pen.gamma, beta)
        got = r["beta_std"][0, l]
        assert np.max(np.abs(got - beta)) <= 1e-8 * max(1e-12, np.abs(beta).max())


def _group_block_cd(Gs, cs, lam, groups):
    p = len(cs)
    beta = np.zeros(p)
    ids = np.unique(groups)
    for _ in range(20000):
        mx = 0.0
        for g in ids:
            m = groups == g
            r = cs[m] - Gs[m] @ beta + Gs[np.ix_(m, m)] @ beta[m]
            lc = lam * math.sqrt(m.sum())
            if np.linalg.norm(r) <= lc:
                nb = np.zeros(m.sum())
            else:
                ev, Q = np.linalg.eigh(Gs[np.ix_(m, m)])
                rh = Q.T @ r
                psi = lambda t: np.sum(rh ** 2 / (ev * t + lc) ** 2) - 1.0
                lo, hi = 0.0, 1.0
                while psi(hi) > 0:
                    hi *= 2
                for _ in range(200):
                    mid = 0.5 * (lo + hi)
                    lo, hi = (mid, hi) if psi(mid) > 0 else (lo, mid)
                t = 0.5 * (lo + hi)
                nb = Q @ (rh / (ev + lc / t))
            mx = max(mx, np.abs(nb - beta[m]).max())
            beta[m] = nb
        if mx <= 1e-14:
            break
    return beta


def test_group_lasso_matches_block_coordinate_descent():
    pr = workloads.cv_grouped(n=3000, p=12, group_size=3, active_groups=2, seed_tag=35)
    st = _stats(pr.X, pr.y)
    groups = pr.groups
    pen = Penalty("grp_lasso")
    lam = oracle.lambda_grid(oracle.lambda_max(st["cs"], pen, groups), 10, 1e-2)
    r = oracle.fit_from_stats(st, [pen], lam[None, :], groups=groups)
    for l in range(1, 10):
        ref = _group_block_cd(st["Gs"], st["cs"], lam[l], groups)
        got = r["beta_std"][0, l]
        assert np.max(np.abs(got - ref)) <= 1e-8 * np.abs(ref).max()
        assert np.array_equal(got != 0, ref != 0)
        # the oracle's group stationarity check: ~0 at the block-descent
        # solution, and the violation of a moved coefficient is at least the
        # change of the gradient in its group less the change of the
        # subgradient direction term (here: a clearly positive value)
        assert oracle.kkt(st["Gs"], st["cs"], pen, lam[l], ref, groups) <= 1e-9 * np.abs(ref).max()
        j = int(np.flatnonzero(ref)[0])
        bad = ref.copy()
        bad[j] += 0.05 * np.abs(ref).max()
        assert oracle.kkt(st["Gs"], st["cs"], pen, lam[l], bad, groups) >= 1e-3 * np.abs(ref).max()


# ------------------------------------------------------------ stationarity, MM

def _kkt_numpy(Gs, cs, beta, lam, kind, alpha=0.5, gamma=3.0):
    g = Gs @ beta - cs
    v = 0.0
    for j in range(len(beta)):
        b = beta[j]
        if b == 0:
            thr = alpha * lam if kind == "enet" else lam
            v = max(v, abs(g[j]) - thr)
            continue
        ab = abs(b)
        dp = {"lasso": lam,
              "enet": alpha * lam + (1 - alpha) * lam * ab,
              "mcp": max(0.0, lam - ab / gamma),
              "scad": lam if ab <= lam else ((gamma * lam - ab) / (gamma - 1) if ab <= gamma * lam else 0.0)}[kind]
        v = max(v, abs(g[j] + np.sign(b) * dp))
    return v


@pytest.mark.parametrize("kind", ["lasso", "enet", "mcp", "scad"])
def test_kkt_at_convergence(kind):
    pr = workloads.small_lasso(seed_tag=36)
    st = _stats(pr.X, pr.y)
    pen = Penalty(kind, alpha=0.5, gamma=3.7 if kind == "scad" else 3.0)
    lam = oracle.lambda_grid(oracle.lambda_max(st["cs"], pen), 50, 1e-3)
    r = oracle.fit_from_stats(st, [pen], lam[None, :])
    assert r["status"] == 0
    for l in range(50):
        b = r["beta_std"][0, l]
        k = _kkt_numpy(st["Gs"], st["cs"], b, lam[l], kind, 0.5, pen.gamma)
        scale = max(np.abs(b).max(), 1e-300)
        # stopping rule: last step moved beta by <= 1e-10 max|beta|; the
        # gradient error is at most about d times that.
        assert k <= 5e-10 * scale * r["d"] + 1e-15
        assert abs(k - r["kkt"][0, l]) <= 1e-12 + 1e-9 * k


@pytest.mark.parametrize("kind", ["lasso", "enet", "mcp", "scad", "grp_lasso"])
def test_each_em_step_does_not_increase_objective(kind):
    pr = workloads.tall_multi(n=5000, p=15, seed_tag=37)
    st = _stats(pr.X, pr.y)
    groups = (np.arange(15) // 3).astype(np.int32)
    pen = Penalty(kind, alpha=0.5, gamma=3.0)
    d = oracle.oem_d(st["Gs"])
    lam = 0.2 * oracle.lambda_max(st["cs"], pen, groups)
    beta, tr = oracle.oem_steps(st["Gs"], st["cs"], st["yyn"], d, pen, lam, np.zeros(15), 60,
                                groups)
    f0 = oracle.objective(st["Gs"], st["cs"], st["yyn"], pen, lam, np.zeros(15), groups)
    seq = np.concatenate([[f0], tr])
    assert np.all(np.diff(seq) <= 1e-14 * np.abs(seq[:-1]))
    assert seq[-1] < seq[0]


def test_objective_formula_matches_residual_form():
    pr = workloads.small_lasso(n=1000, p=6, seed_tag=38)
    st = _stats(pr.X, pr.y, standardize=False)
    beta = np.array([0.3, -0.2, 0.0, 1.1, 0.0, -0.7])
    lam = 0.05
    f = oracle.objective(st["Gs"], st["cs"], st["yyn"], Penalty("lasso"), lam, beta)
    ref = 0.5 * np.mean((pr.y - pr.X @ beta) ** 2) + lam * np.abs(beta).sum()
    assert f == pytest.approx(ref, rel=1e-12)


def test_maxit_flags_nonconvergence():
    pr = workloads.tall_multi(n=2000, p=10, seed_tag=39)
    st = _stats(pr.X, pr.y)
    pen = Penalty("lasso")
    lam = oracle.lambda_grid(oracle.lambda_max(st["cs"], pen), 5, 1e-3)
    r = oracle.fit_path_std(st["Gs"], st["cs"], st["yyn"], oracle.oem_d(st["Gs"]), pen, lam,
                            maxit=2)
    assert r["status"] == 1
    assert r["iters"][0] == 1 and np.all(r["iters"][1:] == -2)


def test_invalid_concavity_rejected():
    st = _stats(*_hadamard_problem())
    with pytest.raises(ValueError):
        oracle.fit_path_std(st["Gs"], st["cs"], st["yyn"], 1.0, Penalty("mcp", gamma=1.0), [0.1])
    with pytest.raises(ValueError):
        oracle.fit_path_std(st["Gs"], st["cs"], st["yyn"], 1.0, Penalty("scad", gamma=2.0), [0.1])
