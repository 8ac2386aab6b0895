"""Pins of the oracle's group MCP, group SCAD and sparse group lasso
(Section 2.2: penalty table, eqs. gmcp, gscad, sglasso).

The penalty values are written here from the penalty table (group MCP and
SCAD read as sum_k P_{lambda c_k, gamma}(||beta_g||): the table's extra
factor lambda is taken as a typo, consistent with the updates).  The pins:

* each group update is the minimiser of d/2 ||b||^2 - u^T b + P(b) (the
  M-step of Section 2.1 restricted to one group), found by brute force;
* special cases that reduce to other penalties: groups of one variable,
  tau = 0 and tau = 1 for the sparse group lasso, gamma -> infinity;
* textbook thresholding rules for an orthonormal design (d = 1);
* the fixed point equals an independent block coordinate descent written
  here (within-group whitened designs, where the block step is closed form)
  for convex instances;
* stationarity at convergence, hand-worked violations at given points, and
  the majorise-minimise property of every EM step.
"""
import math

import numpy as np
import pytest
from scipy import optimize

import oracle
from oracle import Penalty
import workloads


# ------------------------------------------------------------ penalty values

def mcp(t, lc, g):
    return lc * t - t * t / (2 * g) if t <= g * lc else g * lc * lc / 2


def scad(t, lc, g):
    if t <= lc:
        return lc * t
    if t <= g * lc:
        return -(t * t - 2 * g * lc * t + lc * lc) / (2 * (g - 1))
    return (g + 1) * lc * lc / 2


def group_pen(kind, b, cgk, lam, gamma=3.0, tau=0.5, w=None):
    nb = float(np.linalg.norm(b))
    if kind == "grp_mcp":
        return mcp(nb, cgk * lam, gamma)
    if kind == "grp_scad":
        return scad(nb, cgk * lam, gamma)
    if kind == "sgl":
        w = np.ones_like(b) if w is None else w
        return lam * (1 - tau) * cgk * nb + lam * tau * float(np.sum(w * np.abs(b)))
    raise ValueError(kind)


def _soft(z, t):
    return np.sign(z) * np.maximum(np.abs(z) - t, 0.0)


# ------------------------------------------------------------ single-group updates

def _brute_group(h, u, d, rng):
    m = len(u)
    best, bestv = np.zeros(m), h(np.zeros(m))
    starts = [u / d, -u / d, 0.5 * u / d, 1.5 * u / d] + [rng.normal(size=m) for _ in range(2)]
    for s0 in starts:
        r = optimize.minimize(h, s0, method="Nelder-Mead",
                              options=dict(xatol=1e-10, fatol=1e-15, maxiter=6000))
        if r.fun < bestv:
            best, bestv = r.x, r.fun
    if m == 2:      # a grid as well, so a missed basin cannot hide
        span = 2 * np.abs(u).max() / d + 0.5
        t = np.linspace(-span, span, 401)
        for a in t[::4]:
            for b in t[::4]:
                v = h(np.array([a, b]))
                if v < bestv - 1e-9:
                    r = optimize.minimize(h, np.array([a, b]), method="Nelder-Mead",
                                          options=dict(xatol=1e-10, fatol=1e-15))
                    best, bestv = r.x, r.fun
    return best, bestv


CASES = []
_rng = np.random.default_rng(17)
for kind in ["grp_mcp", "grp_scad", "sgl"]:
    for m in [1, 2, 3]:
        for _ in range(4):
            d = float(_rng.uniform(1.2, 3.0))         # d != 1 separates the SGL readings
            lam = float(_rng.uniform(0.05, 0.6))
            cgk = float(_rng.uniform(0.5, 2.0))
            gamma = float(_rng.uniform(2.2, 5.0))
            tau = float(_rng.uniform(0.1, 0.9))
            u = _rng.normal(0, 2.5 * lam * cgk * d, size=m)
            CASES.append((kind, m, d, lam, cgk, gamma, tau, u))


@pytest.mark.parametrize("kind,m,d,lam,cgk,gamma,tau,u", CASES)
def test_group_update_is_minimiser(kind, m, d, lam, cgk, gamma, tau, u):
    pen = Penalty(kind, gamma=gamma, tau=tau)
    got = oracle.prox_group_pen(pen, u, cgk, lam, d)
    h = lambda b: 0.5 * d * b @ b - u @ b + group_pen(kind, b, cgk, lam, gamma, tau)
    best, bestv = _brute_group(h, u, d, np.random.default_rng(m))
    assert h(got) <= bestv + 1e-12
    assert np.max(np.abs(got - best)) <= 1e-5


def test_sgl_printed_composition_is_not_the_minimiser():
    """The printed sparse group lasso step G(S(u, w lambda tau, d), c lambda (1 - tau), 1)
    is the proximal map only when d = 1; with d = 2.5 it lands elsewhere and
    has a larger M-step objective than the oracle's reading."""
    u, d, lam, cgk, tau = np.array([1.3, -0.4]), 2.5, 0.3, math.sqrt(2), 0.4
    pen = Penalty("sgl", tau=tau)
    ours = oracle.prox_group_pen(pen, u, cgk, lam, d)
    v = _soft(u, lam * tau) / d
    nv = np.linalg.norm(v)
    printed = v * max(0.0, 1 - cgk * lam * (1 - tau) / nv)
    h = lambda b: 0.5 * d * b @ b - u @ b + group_pen("sgl", b, cgk, lam, tau=tau)
    assert np.abs(ours - printed).max() > 1e-3
    assert h(ours) < h(printed) - 1e-6


def test_group_updates_zero_and_scaling():
    for kind in ["grp_mcp", "grp_scad", "sgl"]:
        pen = Penalty(kind, gamma=3.5, tau=0.3)
        assert np.array_equal(oracle.prox_group_pen(pen, np.zeros(3), 1.0, 0.2, 1.4), np.zeros(3))
        # inside the dead zone the whole group is zero
        u = np.array([0.05, -0.02, 0.01])
        assert np.array_equal(oracle.prox_group_pen(pen, u, 1.0, 0.2, 1.4), np.zeros(3))
        # lambda = 0: plain division by d
        u = np.array([0.7, -0.2])
        assert np.allclose(oracle.prox_group_pen(pen, u, 1.0, 0.0, 1.4), u / 1.4, rtol=1e-15)
    # group MCP / SCAD keep the direction of u (radial updates, eqs. gmcp, gscad)
    u = np.array([1.0, -2.0, 0.5])
    for kind in ["grp_mcp", "grp_scad"]:
        out = oracle.prox_group_pen(Penalty(kind, gamma=3.0), u, 1.0, 0.4, 1.2)
        assert np.allclose(out / np.linalg.norm(out), u / np.linalg.norm(u), rtol=0, atol=1e-15)


def test_group_update_hand_worked():
    """Values worked by hand from eqs. gmcp, gscad and the sparse group
    lasso's nested thresholding, u = (3, 4), ||u|| = 5, c_k = 1, d = 2."""
    u = np.array([3.0, 4.0])
    # group MCP, lambda = 1, gamma = 3: ||u|| = 5 <= gamma lambda d = 6, so
    # t = gamma (5 - 1) / (gamma d - 1) = 12 / 5 = 2.4, beta = 2.4 (0.6, 0.8)
    got = oracle.prox_group_pen(Penalty("grp_mcp", gamma=3.0), u, 1.0, 1.0, 2.0)
    assert np.allclose(got, [1.44, 1.92], rtol=1e-15)
    # ||u|| = 5 > 6?  no; with lambda = 0.8, gamma lambda d = 4.8 < 5: u / d
    got = oracle.prox_group_pen(Penalty("grp_mcp", gamma=3.0), u, 1.0, 0.8, 2.0)
    assert np.allclose(got, [1.5, 2.0], rtol=1e-15)
    # group SCAD, gamma = 3.7, lambda = 1: (d + 1) lambda = 3 < 5 <= 7.4, so
    # t = ((gamma - 1) 5 - gamma) / ((gamma - 1) d - 1) = 9.8 / 4.4
    got = oracle.prox_group_pen(Penalty("grp_scad", gamma=3.7), u, 1.0, 1.0, 2.0)
    t = 9.8 / 4.4
    assert np.allclose(got, [0.6 * t, 0.8 * t], rtol=1e-14)
    # group SCAD, lambda = 2: 5 <= (d + 1) lambda = 6, soft region: (5 - 2) / 2 = 1.5
    got = oracle.prox_group_pen(Penalty("grp_scad", gamma=3.7), u, 1.0, 2.0, 2.0)
    assert np.allclose(got, [0.9, 1.2], rtol=1e-15)
    # sparse group lasso, tau = 0.5, lambda = 2: v = soft(u, 1) = (2, 3),
    # ||v|| = sqrt(13), factor 1 - 1 / sqrt(13), beta = (v / 2) factor
    got = oracle.prox_group_pen(Penalty("sgl", tau=0.5), u, 1.0, 2.0, 2.0)
    f = 1 - 1 / math.sqrt(13)
    assert np.allclose(got, [1.0 * f, 1.5 * f], rtol=1e-15)


# ------------------------------------------------------------ paths

def _problem(n=3000, p=20, group_size=4, seed_tag=71, rho=0.4):
    pr = workloads.cv_grouped(n=n, p=p, group_size=group_size, active_groups=2,
                              seed_tag=seed_tag, rho=rho)
    G, b, yy, nn = oracle.gram_train(pr.X, pr.y, -1)
    st = oracle.prepare(G, b, yy, nn, True)
    return pr, st


def _fit(st, pen, lam, groups, d=None, tol=1e-12, w=None, cg=None):
    return oracle.fit_from_stats(st, [pen], lam[None, :] if lam.ndim == 1 else lam, groups,
                                 w, cg, tol=tol, maxit=500000, d=d)


def test_singleton_groups_reduce_to_scalar_penalties():
    """Groups of one variable (c_k = 1): group MCP is MCP, group SCAD is SCAD,
    the sparse group lasso is the lasso for any tau."""
    pr, st = _problem()
    p = len(st["cs"])
    groups = np.arange(p, dtype=np.int32)
    lam = oracle.lambda_grid(oracle.lambda_max(st["cs"], Penalty("lasso")), 15, 0.02)
    for gk, sk in [(Penalty("grp_mcp", gamma=3.0), Penalty("mcp", gamma=3.0)),
                   (Penalty("grp_scad", gamma=3.7), Penalty("scad", gamma=3.7)),
                   (Penalty("sgl", tau=0.35), Penalty("lasso"))]:
        a = _fit(st, gk, lam, groups)["beta_std"][0]
        b = _fit(st, sk, lam, None)["beta_std"][0]
        for l in range(len(lam)):
            s = np.abs(b[l]).max()
            assert np.abs(a[l] - b[l]).max() <= 1e-11 * max(s, 1e-300), (gk.kind, l)
            assert np.array_equal(a[l] != 0, b[l] != 0)


def test_sgl_endpoints():
    """tau = 0 is the group lasso, tau = 1 the lasso (groups of four)."""
    pr, st = _problem()
    groups = pr.groups
    lam = oracle.lambda_grid(oracle.lambda_max(st["cs"], Penalty("grp_lasso"), groups), 15, 0.02)
    a = _fit(st, Penalty("sgl", tau=0.0), lam, groups)["beta_std"][0]
    b = _fit(st, Penalty("grp_lasso"), lam, groups)["beta_std"][0]
    assert np.array_equal(a, b)
    lam = oracle.lambda_grid(oracle.lambda_max(st["cs"], Penalty("lasso")), 15, 0.02)
    a = _fit(st, Penalty("sgl", tau=1.0), lam, groups)["beta_std"][0]
    b = _fit(st, Penalty("lasso"), lam, None)["beta_std"][0]
    for l in range(len(lam)):
        assert np.abs(a[l] - b[l]).max() <= 1e-12 * max(np.abs(b[l]).max(), 1e-300)


def test_group_mcp_large_gamma_is_group_lasso():
    pr, st = _problem()
    groups = pr.groups
    lam = oracle.lambda_grid(oracle.lambda_max(st["cs"], Penalty("grp_lasso"), groups), 12, 0.05)
    a = _fit(st, Penalty("grp_mcp", gamma=1e9), lam, groups)["beta_std"][0]
    b = _fit(st, Penalty("grp_lasso"), lam, groups)["beta_std"][0]
    for l in range(1, len(lam)):
        assert np.abs(a[l] - b[l]).max() <= 1e-6 * np.abs(b[l]).max()
        assert np.array_equal(a[l] != 0, b[l] != 0)


def _hadamard(p=8, n=64, seed=11):
    H = np.array([[1.0]])
    while H.shape[0] < n:
        H = np.block([[H, H], [H, -H]])
    X = np.ascontiguousarray(H[:, 1:p + 1])
    rng = np.random.default_rng(seed)
    y = X @ rng.normal(0, 1.0, size=p) + rng.normal(0, 0.5, size=n)
    return X, y


def _firm(z, lc, g):       # textbook firm thresholding (d = 1)
    return 0.0 if z <= lc else (g * (z - lc) / (g - 1) if z <= g * lc else z)


def _fanli(z, lc, a):      # Fan & Li (2001) SCAD rule (d = 1)
    if z <= 2 * lc:
        return max(z - lc, 0.0)
    if z <= a * lc:
        return ((a - 1) * z - a * lc) / (a - 2)
    return z


@pytest.mark.parametrize("kind", ["grp_mcp", "grp_scad", "sgl"])
def test_orthonormal_design_closed_forms(kind):
    """X^T X / n = I: with d = 1 the fixed point is the textbook rule applied
    to c (firm and Fan-Li thresholding of ||c_g||; for the sparse group lasso
    the group soft threshold of soft(c, lambda tau))."""
    X, y = _hadamard()
    G, b, yy, n = oracle.gram_train(X, y, -1)
    st = oracle.prepare(G, b, yy, n, True)
    assert np.allclose(st["Gs"], np.eye(8), atol=0)
    groups = np.array([0, 0, 1, 1, 1, 2, 3, 3], dtype=np.int32)
    cgs = np.sqrt(np.bincount(groups))
    c = st["cs"]
    pen = Penalty(kind, gamma=3.7, tau=0.4)
    lmax = oracle.lambda_max(c, pen, groups)
    lam = oracle.lambda_grid(lmax, 10, 0.05)
    res = _fit(st, pen, lam, groups, d=1.0)["beta_std"][0]
    for l, lv in enumerate(lam):
        want = np.zeros(8)
        for g in range(4):
            m = groups == g
            if kind == "sgl":
                v = _soft(c[m], lv * 0.4)
                nv = np.linalg.norm(v)
                want[m] = v * max(0.0, 1 - lv * 0.6 * cgs[g] / nv) if nv > 0 else 0.0
            else:
                z = np.linalg.norm(c[m])
                t = _firm(z, lv * cgs[g], 3.7) if kind == "grp_mcp" else _fanli(z, lv * cgs[g], 3.7)
                want[m] = t * c[m] / z
        assert np.allclose(res[l], want, rtol=1e-12, atol=1e-14), (kind, l)


def _whitened_groups(st, groups):
    """The same problem with each group's columns whitened (G_gg = I): the
    block coordinate descent step then has a closed form."""
    Gs, cs = st["Gs"], st["cs"]
    p = len(cs)
    T = np.zeros((p, p))
    for g in np.unique(groups):
        m = np.nonzero(groups == g)[0]
        ev, V = np.linalg.eigh(Gs[np.ix_(m, m)])
        T[np.ix_(m, m)] = V @ np.diag(ev ** -0.5) @ V.T
    G2 = T @ Gs @ T
    G2 = 0.5 * (G2 + G2.T)
    for g in np.unique(groups):
        m = np.nonzero(groups == g)[0]
        G2[np.ix_(m, m)] = np.eye(len(m))
    return dict(Gs=G2, cs=T @ cs, yyn=st["yyn"], s=np.ones(p))


def _bcd(G, c, groups, cgs, kind, lam, gamma, tau, beta0, sweeps=20000):
    beta = beta0.copy()
    ids = [np.nonzero(groups == g)[0] for g in range(groups.max() + 1)]
    for _ in range(sweeps):
        old = beta.copy()
        for g, m in enumerate(ids):
            z = c[m] - G[m] @ beta + beta[m]          # G_gg = I
            if kind == "sgl":
                v = _soft(z, lam * tau)
                nv = np.linalg.norm(v)
                beta[m] = v * max(0.0, 1 - lam * (1 - tau) * cgs[g] / nv) if nv > 0 else 0.0
            else:
                nz = np.linalg.norm(z)
                t = _firm(nz, lam * cgs[g], gamma) if kind == "grp_mcp" else _fanli(nz, lam * cgs[g], gamma)
                beta[m] = t * z / nz if nz > 0 else 0.0
        if np.abs(beta - old).max() <= 1e-15 * max(np.abs(beta).max(), 1e-300):
            break
    return beta


@pytest.mark.parametrize("kind,gamma,tau", [("sgl", 3.0, 0.3), ("grp_mcp", 6.0, 0.0),
                                            ("grp_scad", 6.0, 0.0)])
def test_fixed_point_equals_block_coordinate_descent(kind, gamma, tau):
    """Convex instances (sparse group lasso; group MCP / SCAD with gamma
    large enough that G - I / gamma (MCP) or G - I / (gamma - 1) (SCAD) is
    positive definite): the minimiser is unique, so OEM's fixed point equals
    the block coordinate descent solution."""
    pr, st0 = _problem(p=16, group_size=4, seed_tag=73, rho=0.3)
    groups = pr.groups
    st = _whitened_groups(st0, groups)
    lam_min = float(np.linalg.eigvalsh(st["Gs"]).min())
    assert lam_min > 1.0 / (gamma - 1.0)
    cgs = np.sqrt(np.bincount(groups))
    pen = Penalty(kind, gamma=gamma, tau=tau)
    lam = oracle.lambda_grid(oracle.lambda_max(st["cs"], pen, groups), 10, 0.05)
    res = _fit(st, pen, lam, groups, tol=1e-13)
    beta = np.zeros(len(st["cs"]))
    for l, lv in enumerate(lam):
        beta = _bcd(st["Gs"], st["cs"], groups, cgs, kind, lv, gamma, tau, beta)
        got = res["beta_std"][0, l]
        s = max(np.abs(beta).max(), 1e-300)
        assert np.abs(got - beta).max() <= 1e-9 * s, (kind, l)
        assert np.array_equal(got != 0, beta != 0)


@pytest.mark.parametrize("kind", ["grp_mcp", "grp_scad", "sgl"])
def test_kkt_at_convergence_and_mm(kind):
    pr, st = _problem(p=24, group_size=4, seed_tag=74)
    groups = pr.groups
    pen = Penalty(kind, gamma=3.0 if kind != "grp_scad" else 3.7, tau=0.3)
    lam = oracle.lambda_grid(oracle.lambda_max(st["cs"], pen, groups), 20, 0.01)
    res = _fit(st, pen, lam, groups)
    assert np.all(res["kkt"][0] <= 1e-8)
    assert res["beta_std"][0, 0].max() == 0.0 and res["beta_std"][0, 0].min() == 0.0
    assert np.any(res["beta_std"][0, 1] != 0)          # lambda_max is the smallest zero level
    # every EM step decreases the objective (majorise-minimise, Section 2.1)
    d = res["d"]
    _, tr = oracle.oem_steps(st["Gs"], st["cs"], st["yyn"], d, pen, lam[8],
                             res["beta_std"][0, 4], 60, groups)
    assert np.all(np.diff(tr) <= 1e-13 * np.abs(tr).max())


def test_lambda_max_is_the_smallest_zero_level():
    pr, st = _problem(p=24, group_size=4, seed_tag=75)
    groups = pr.groups
    cgs = np.sqrt(np.bincount(groups))
    for pen in [Penalty("grp_mcp", gamma=3.0), Penalty("grp_scad", gamma=3.7),
                Penalty("sgl", tau=0.25), Penalty("sgl", tau=0.8), Penalty("sgl", tau=1.0)]:
        lm = oracle.lambda_max(st["cs"], pen, groups)
        for lv, zero in [(lm, True), (lm * (1 - 1e-9), False)]:
            out = np.concatenate([oracle.prox_group_pen(pen, st["cs"][groups == g], cgs[g], lv, 1.0)
                                  for g in range(groups.max() + 1)])
            assert np.all(out == 0.0) == zero, (pen, lv)
    # group MCP / SCAD: max_g ||c_g|| / c_g; sparse group lasso tau = 1: max |c_j|
    c = st["cs"]
    want = max(np.linalg.norm(c[groups == g]) / cgs[g] for g in range(groups.max() + 1))
    assert oracle.lambda_max(c, Penalty("grp_mcp", gamma=3.0), groups) == pytest.approx(want, rel=1e-15)
    assert oracle.lambda_max(c, Penalty("sgl", tau=1.0), groups) == pytest.approx(np.abs(c).max(), rel=1e-15)


def test_kkt_hand_worked():
    """G = [[1, .5], [.5, 1]], c = (.9, -.3), one group of two (c_k = sqrt 2),
    lambda = 0.2.  At beta = 0 the gradient is -c, ||c|| = sqrt(0.9):
    group MCP / SCAD violation sqrt(0.9) - 0.2 sqrt 2; sparse group lasso
    (tau = 0.5) ||soft(c, 0.1)|| - 0.1 sqrt 2 = sqrt(0.68) - 0.1 sqrt 2.
    At beta = (0.5, 0): gradient (-0.4, 0.55); group MCP (gamma = 3)
    P'(0.5) = 0.2 sqrt 2 - 0.5 / 3, residual (-0.4 + P'(0.5), 0.55)."""
    Gs = np.array([[1.0, 0.5], [0.5, 1.0]])
    cs = np.array([0.9, -0.3])
    groups = np.array([0, 0], dtype=np.int32)
    r2 = math.sqrt(2.0)
    z = np.zeros(2)
    assert oracle.kkt(Gs, cs, Penalty("grp_mcp", gamma=3.0), 0.2, z, groups) == pytest.approx(
        math.sqrt(0.9) - 0.2 * r2, rel=1e-14)
    assert oracle.kkt(Gs, cs, Penalty("grp_scad", gamma=3.7), 0.2, z, groups) == pytest.approx(
        math.sqrt(0.9) - 0.2 * r2, rel=1e-14)
    assert oracle.kkt(Gs, cs, Penalty("sgl", tau=0.5), 0.2, z, groups) == pytest.approx(
        math.sqrt(0.68) - 0.1 * r2, rel=1e-14)
    b = np.array([0.5, 0.0])
    dp = 0.2 * r2 - 0.5 / 3.0
    want = math.hypot(-0.4 + dp, 0.55)
    assert oracle.kkt(Gs, cs, Penalty("grp_mcp", gamma=3.0), 0.2, b, groups) == pytest.approx(want, rel=1e-14)
    # sparse group lasso at beta = (0.5, 0), tau = 0.5: member 0 residual
    # -0.4 + 0.1 sqrt 2 + 0.1; member 1 (zero) max(|0.55| - 0.1, 0) = 0.45
    want = math.hypot(-0.4 + 0.1 * r2 + 0.1, 0.45)
    assert oracle.kkt(Gs, cs, Penalty("sgl", tau=0.5), 0.2, b, groups) == pytest.approx(want, rel=1e-14)
    # objective at beta = (0.5, 0): 1/2 b^T G b - c^T b = 0.125 - 0.45, plus
    # group MCP P(0.5) = 0.2 sqrt 2 * 0.5 - 0.25 / 6 (0.5 <= 3 * 0.2 sqrt 2)
    f = oracle.objective(Gs, cs, 0.0, Penalty("grp_mcp", gamma=3.0), 0.2, b, groups)
    assert f == pytest.approx(0.125 - 0.45 + 0.1 * r2 - 0.25 / 6.0, rel=1e-14)
    # group SCAD (gamma = 3.7): lambda c = 0.2 sqrt 2 < 0.5 <= 3.7 * 0.2 sqrt 2,
    # P = -(0.25 - 2 * 3.7 * 0.2 sqrt 2 * 0.5 + 0.08) / (2 * 2.7)
    f = oracle.objective(Gs, cs, 0.0, Penalty("grp_scad", gamma=3.7), 0.2, b, groups)
    assert f == pytest.approx(0.125 - 0.45 - (0.25 - 0.74 * r2 + 0.08) / 5.4, rel=1e-14)
    # sparse group lasso (tau = 0.5): 0.2 * 0.5 * sqrt 2 * 0.5 + 0.2 * 0.5 * 0.5
    f = oracle.objective(Gs, cs, 0.0, Penalty("sgl", tau=0.5), 0.2, b, groups)
    assert f == pytest.approx(0.125 - 0.45 + 0.05 * r2 + 0.05, rel=1e-14)
