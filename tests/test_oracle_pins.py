"""Literal pins of the oracle's lambda sequence, group stationarity check and
CV selection: every expected value below is written out by hand (exact
binary fractions, or a closed form evaluated once), so a slip in the
oracle's arithmetic (an exponent l/L instead of l/(L-1), a dropped term of
the group subgradient, a wrong denominator in cvsd) fails here.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import Penalty


# ------------------------------------------------------------ lambda sequence

def test_lambda_grid_endpoints_and_spacing_literal():
    # lambda_max = 2, ratio 1e-2, L = 5: 2 * 10^(-2 l / 4)
    got = oracle.lambda_grid(2.0, 5, 1e-2)
    want = [2.0, 0.6324555320336759, 0.2, 0.06324555320336758, 0.02]
    assert got[0] == 2.0                    # lambda_1 = lambda_max exactly
    assert got[-1] == pytest.approx(0.02, rel=2e-16, abs=0)
    for g, w in zip(got, want):
        assert g == pytest.approx(w, rel=4e-16, abs=0)
    # constant log spacing: every ratio of neighbours is 10^-0.5
    r = got[1:] / got[:-1]
    assert np.all(np.abs(r - 0.31622776601683794) <= 4e-16)


def test_lambda_grid_short_sequences():
    assert list(oracle.lambda_grid(3.5, 1, 1e-3)) == [3.5]
    two = oracle.lambda_grid(3.5, 2, 1e-3)
    assert two[0] == 3.5 and two[1] == pytest.approx(3.5e-3, rel=2e-16, abs=0)


@pytest.mark.parametrize("kind,extra,want", [
    ("lasso", {}, 0.7),
    ("mcp", dict(gamma=3.0), 0.7),
    ("scad", dict(gamma=3.7), 0.7),
    ("enet", dict(alpha=0.5), 1.4),
    ("enet", dict(alpha=0.25), 2.8),
])
def test_lambda_max_separable_literal(kind, extra, want):
    cs = np.array([0.3, -0.7, 0.5])
    got = oracle.lambda_max(cs, Penalty(kind, **extra))
    # the smallest lambda whose update maps beta = 0 to 0: max |c_j| / (w_j a)
    # (a = alpha for the elastic net), up to the few ulps it may be raised
    assert got == pytest.approx(want, rel=1e-15, abs=0)


def test_lambda_max_weights_literal():
    cs = np.array([0.3, -0.7, 0.5])
    w = np.array([1.0, 2.0, 0.0])         # w = 0: unpenalised, never limits lambda
    got = oracle.lambda_max(cs, Penalty("lasso"), w=w)
    assert got == pytest.approx(0.35, rel=1e-15, abs=0)   # max(0.3 / 1, 0.7 / 2)


def test_lambda_max_group_literal():
    cs = np.array([0.3, -0.7, 0.5])
    groups = np.array([0, 0, 1], dtype=np.int32)
    # groups {0, 1} (c = sqrt 2) and {2} (c = 1): max(sqrt(0.58) / sqrt 2, 0.5)
    got = oracle.lambda_max(cs, Penalty("grp_lasso"), groups)
    assert got == pytest.approx(0.5385164807134504, rel=1e-15, abs=0)


# ------------------------------------------------------------ group stationarity

def _grp_problem():
    # orthonormal design: Gs = I, cs = (3, 4), one group of two, c = sqrt 2
    return np.eye(2), np.array([3.0, 4.0]), np.array([0, 0], dtype=np.int32)


def test_group_kkt_literal_values():
    Gs, cs, groups = _grp_problem()
    pen = Penalty("grp_lasso")
    lam = 1.0
    # beta = 0: gradient -cs, violation ||cs|| - lambda c = 5 - sqrt 2
    v0 = oracle.kkt(Gs, cs, pen, lam, np.zeros(2), groups)
    assert v0 == pytest.approx(3.585786437626905, rel=1e-15)
    # beta along cs with norm 1/2: residual (||beta|| - ||cs|| + lambda c) cs/||cs||
    v1 = oracle.kkt(Gs, cs, pen, lam, np.array([0.3, 0.4]), groups)
    assert v1 == pytest.approx(3.085786437626905, rel=1e-15)
    # beta off the direction of cs: |(0.4 - 3 + 0.8 sqrt 2, 0.3 - 4 + 0.6 sqrt 2)|
    v2 = oracle.kkt(Gs, cs, pen, lam, np.array([0.4, 0.3]), groups)
    assert v2 == pytest.approx(3.2074543431811127, rel=1e-15)
    # the group soft-threshold of cs is the minimiser: no violation
    star = cs * (1.0 - math.sqrt(2.0) / 5.0)
    assert oracle.kkt(Gs, cs, pen, lam, star, groups) <= 1e-15
    # a zero group whose gradient norm is below lambda c is stationary
    assert oracle.kkt(Gs, cs, pen, 6.0 / math.sqrt(2.0), np.zeros(2), groups) == 0.0


def test_group_objective_literal():
    Gs, cs, groups = _grp_problem()
    # f = 1/2 b'b - c'b + 1/2 yy/n + lambda c ||b||, b = (0.3, 0.4), yy/n = 2
    f = oracle.objective(Gs, cs, 2.0, Penalty("grp_lasso"), 1.0, np.array([0.3, 0.4]), groups)
    want = 0.5 * 0.25 - (0.9 + 1.6) + 1.0 + math.sqrt(2.0) * 0.5
    assert f == pytest.approx(want, rel=1e-15)


# ------------------------------------------------------------ CV selection

def _hand_mse():
    # two penalties, K = 3 folds of sizes 1, 1, 2 (weights 1/4, 1/4, 1/2), L = 4
    mse = np.array([
        [[2.0, 2.0, 1.0, 3.0], [2.0, 2.0, 3.0, 3.0], [1.5, 1.0, 2.0, 3.0]],
        [[3.0, 1.0, 1.0, 2.0], [3.0, 2.0, 1.0, 2.0], [3.0, 1.0, 1.5, 2.0]],
    ])
    return mse, np.array([1, 1, 2], dtype=np.int64)


def test_select_literal_values():
    mse, nk = _hand_mse()
    s = oracle.select(mse, nk)
    # cvm_l = sum_k n_k MSE_kl / n, n = 4
    assert list(s["cvm"][0]) == [1.75, 1.5, 2.0, 3.0]
    assert list(s["cvm"][1]) == [3.0, 1.25, 1.25, 2.0]
    # cvsd_l = sqrt(sum_k n_k (MSE_kl - cvm_l)^2 / (n (K - 1))), n (K - 1) = 8
    want0 = [0.1767766952966369, 0.3535533905932738, 0.5, 0.0]    # sqrt(1/32), sqrt(1/8), sqrt(1/4)
    want1 = [0.0, 0.30618621784789724, 0.1767766952966369, 0.0]   # sqrt(3/32), sqrt(1/32)
    assert np.allclose(s["cvsd"][0], want0, rtol=1e-15, atol=0)
    assert np.allclose(s["cvsd"][1], want1, rtol=1e-15, atol=0)
    # lambda_min: argmin; penalty 1 ties at l = 1, 2 -> the larger lambda (1)
    assert list(s["i_min"]) == [1, 1]
    # lambda_1se: first (largest) lambda with cvm <= cvm_min + cvsd_min:
    # penalty 0 threshold 1.5 + sqrt(1/8) = 1.854 takes l = 0 (1.75)
    assert list(s["i_1se"]) == [0, 1]
    assert s["best"] == 1                  # min cvm 1.25 < 1.5


def test_select_i_1se_is_not_argmin_neighbour():
    # the 1-SE rule scans from the largest lambda: a far earlier index qualifies
    mse = np.array([[[1.0, 5.0, 0.75, 0.5], [1.0, 5.0, 0.75, 1.5]]])
    nk = np.array([2, 2], dtype=np.int64)
    s = oracle.select(mse, nk)
    assert list(s["cvm"][0]) == [1.0, 5.0, 0.75, 1.0]
    assert s["i_min"][0] == 2 and s["cvsd"][0][2] == 0.0
    # threshold 0.75: only l = 2 qualifies
    assert s["i_1se"][0] == 2
    mse[0, 1, 2] = 1.25        # cvm_2 = 1.0 ties l = 0 and 3; cvsd_2 = sqrt(2 * 0.0625 * 2 / 4)
    s = oracle.select(mse, nk)
    assert s["cvm"][0][2] == 1.0 and s["i_min"][0] == 0     # tie -> first index
    assert s["i_1se"][0] == 0
