"""Pins of the oracle's thresholding operators (Section 2.2).

Each scalar update must be the minimiser of  d/2 b^2 - u b + P(b)  (the
coordinate-wise M-step of Section 2.1 with A = d I - X^T X).  The penalty
values below are written from the penalty table, and the minimiser is found by
brute force, independently of the closed-form updates.
"""
import math

import numpy as np
import pytest
from scipy import optimize

import oracle
from oracle import Penalty


def pen_value(kind, b, lw, alpha=1.0, gamma=3.0):
    ab = abs(b)
    if kind == "lasso":
        return lw * ab
    if kind == "enet":
        return alpha * lw * ab + 0.5 * (1 - alpha) * lw * b * b
    if kind == "mcp":
        return lw * ab - b * b / (2 * gamma) if ab <= gamma * lw else gamma * lw * lw / 2
    if kind == "scad":
        if ab <= lw:
            return lw * ab
        if ab <= gamma * lw:
            return -(ab * ab - 2 * gamma * lw * ab + lw * lw) / (2 * (gamma - 1))
        return (gamma + 1) * lw * lw / 2
    raise ValueError(kind)


def brute_min(u, lw, d, kind, alpha=1.0, gamma=3.0):
    h = lambda b: 0.5 * d * b * b - u * b + pen_value(kind, b, lw, alpha, gamma)
    span = 2 * abs(u) / d + 1.0
    grid = np.linspace(-span, span, 400_001)
    hv = 0.5 * d * grid * grid - u * grid + np.vectorize(
        lambda b: pen_value(kind, b, lw, alpha, gamma))(grid)
    i = int(np.argmin(hv))
    lo, hi = grid[max(0, i - 2)], grid[min(len(grid) - 1, i + 2)]
    r = optimize.minimize_scalar(h, bounds=(lo, hi), method="bounded",
                                 options=dict(xatol=1e-13))
    best = r.x if h(r.x) <= h(grid[i]) else grid[i]
    if h(0.0) <= h(best):
        best = 0.0
    return best


CASES = []
_rng = np.random.default_rng(5)
for kind in ["lasso", "enet", "mcp", "scad"]:
    for _ in range(12):
        d = float(_rng.uniform(1.0, 3.0))
        lw = float(_rng.uniform(0.05, 1.0))
        u = float(_rng.normal(0, 3 * lw * d))
        alpha = float(_rng.uniform(0.2, 1.0))
        gamma = float(_rng.uniform(2.1, 5.0))
        CASES.append((kind, u, lw, d, alpha, gamma))


@pytest.mark.parametrize("kind,u,lw,d,alpha,gamma", CASES)
def test_scalar_update_is_minimiser(kind, u, lw, d, alpha, gamma):
    pen = Penalty(kind, alpha=alpha, gamma=gamma)
    got = oracle.prox1(pen, u, lw, d)
    ref = brute_min(u, lw, d, kind, alpha, gamma)
    assert abs(got - ref) <= 2e-7 * max(1.0, abs(ref))
    h = lambda b: 0.5 * d * b * b - u * b + pen_value(kind, b, lw, alpha, gamma)
    assert h(got) <= h(ref) + 1e-12


@pytest.mark.parametrize("kind", ["mcp", "scad"])
def test_updates_continuous_at_region_boundaries(kind):
    d, lw, g = 1.7, 0.3, 3.7
    pen = Penalty(kind, gamma=g)
    edges = [lw * g * d] + ([(d + 1) * lw] if kind == "scad" else [])
    for e in edges:
        lo = oracle.prox1(pen, e * (1 - 1e-12), lw, d)
        hi = oracle.prox1(pen, e * (1 + 1e-12), lw, d)
        assert abs(lo - hi) <= 1e-10


def test_zero_input_and_sign_symmetry():
    for kind in ["lasso", "enet", "mcp", "scad"]:
        pen = Penalty(kind, alpha=0.5, gamma=3.0)
        assert oracle.prox1(pen, 0.0, 0.2, 1.5) == 0.0
        for u in [0.1, 0.7, 3.0]:
            assert oracle.prox1(pen, -u, 0.2, 1.5) == -oracle.prox1(pen, u, 0.2, 1.5)


def test_lambda_zero_is_plain_division():
    for kind in ["lasso", "enet", "mcp", "scad"]:
        pen = Penalty(kind, alpha=0.5, gamma=3.0)
        assert oracle.prox1(pen, 0.37, 0.0, 1.3) == pytest.approx(0.37 / 1.3, rel=1e-15)


@pytest.mark.parametrize("m,seed", [(1, 0), (2, 1), (3, 2), (2, 3)])
def test_group_update_is_minimiser(m, seed):
    rng = np.random.default_rng(seed)
    d = float(rng.uniform(1.0, 2.5))
    lc = float(rng.uniform(0.1, 1.0))
    u = rng.normal(0, 1.5 * lc * d, size=m)
    h = lambda b: 0.5 * d * b @ b - u @ b + lc * np.linalg.norm(b)
    got = oracle.prox_group(u, lc, d)
    best, bestv = np.zeros(m), h(np.zeros(m))
    for start in [u / d, -u / d, rng.normal(size=m), 0.5 * u / d]:
        r = optimize.minimize(h, start, method="Nelder-Mead",
                              options=dict(xatol=1e-12, fatol=1e-15, maxiter=20000))
        if r.fun < bestv:
            best, bestv = r.x, r.fun
    assert h(got) <= bestv + 1e-12
    assert np.max(np.abs(got - best)) <= 1e-5


def test_group_zero_norm_gives_zero():
    assert np.array_equal(oracle.prox_group(np.zeros(4), 0.3, 1.2), np.zeros(4))
