"""Pins of the oracle's fold hash, Gram sums and eigenvalue solver.

Each check compares the oracle with something other than itself: a published
generator output, an independent numpy implementation of the published
generator, exact integer arithmetic, closed-form spectra, or a library
eigen-solver.
"""
import math
import os

import numpy as np
import pytest
from scipy import stats

import oracle
import workloads

MASK = (1 << 64) - 1


def _np_splitmix_fold(seed: int, n: int, K: int, row_offset: int = 0) -> np.ndarray:
    """Independent numpy SplitMix64: state_i = seed + (i+1) * golden, then mix."""
    with np.errstate(over="ignore"):
        i = np.arange(row_offset + 1, row_offset + n + 1, dtype=np.uint64)
        z = np.uint64(seed & MASK) + i * np.uint64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
        hi = z >> np.uint64(32)
        return ((hi * np.uint64(K)) >> np.uint64(32)).astype(np.uint8)


def test_splitmix64_published_outputs(golden_dir):
    lines = [l.split() for l in open(os.path.join(golden_dir, "splitmix64_seed1234567.txt"))
             if l.strip() and not l.startswith("#")]
    seed = int(lines[0][1])
    expected = [int(l[0]) for l in lines[1:]]
    assert oracle.splitmix64(seed, len(expected)) == expected


@pytest.mark.parametrize("K", [2, 5, 7, 10])
@pytest.mark.parametrize("seed", [0, 180109661, 2**63 + 12345])
def test_fold_hash_bit_exact_vs_numpy(K, seed):
    n = 50_000
    off = 123_456_789
    assert np.array_equal(oracle.fold_ids(seed, n, K, off), _np_splitmix_fold(seed, n, K, off))


def test_fold_hash_uniform():
    K, n = 10, 1_000_000
    f = oracle.fold_ids(42, n, K)
    counts = np.bincount(f, minlength=K)
    assert counts.sum() == n and f.max() < K
    chi2 = ((counts - n / K) ** 2 / (n / K)).sum()
    assert stats.chi2.sf(chi2, K - 1) > 1e-4


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_gram_integer_exact(dtype):
    """Integer X in [-8, 8]: every product and partial sum is an exact integer."""
    n, p, K = 3000, 13, 4
    X = workloads.integer_rows(n, p, dtype=dtype)
    y = workloads.integer_response(n)
    G, b, yy, nk = oracle.gram_folds(X, y, K, fold_seed=7)
    f = _np_splitmix_fold(7, n, K)
    Xi = X.astype(np.int64)
    yi = y.astype(np.int64)
    for k in range(K):
        m = f == k
        assert np.array_equal(G[k], (Xi[m].T @ Xi[m]).astype(np.float64))
        assert np.array_equal(b[k], (Xi[m].T @ yi[m]).astype(np.float64))
        assert yy[k] == float((yi[m] ** 2).sum())
        assert nk[k] == m.sum()
    Gf, bf, yyf, nf = oracle.gram_train(X, y, -1)
    assert np.array_equal(G.sum(axis=0), Gf) and np.array_equal(b.sum(axis=0), bf)
    assert nf == n and yyf == yy.sum()
    for k in range(K):
        Gt, bt, yyt, nt = oracle.gram_train(X, y, k, K, fold_seed=7)
        others = [c for c in range(K) if c != k]
        assert np.array_equal(Gt, G[others].sum(axis=0))
        assert nt == n - nk[k]


def _sylvester(m: int) -> np.ndarray:
    H = np.array([[1.0]])
    while H.shape[0] < m:
        H = np.block([[H, H], [H, -H]])
    return H


def test_gram_hadamard_is_scaled_identity():
    H = _sylvester(64)
    X = np.ascontiguousarray(H[:, :16]).astype(np.float32)
    G, b, yy, nk = oracle.gram_folds(X, np.ones(64), 1)
    assert np.array_equal(G[0], 64.0 * np.eye(16))


def test_gram_random_within_rounding_bound():
    n, p = 20_000, 9
    X = workloads.draw_rows(n, p, 0.5, np.float32, workloads.subseed(900))
    y = np.ones(n)
    G, _, _, _ = oracle.gram_folds(X, y, 1)
    Xl = X.astype(np.longdouble)
    exact = (Xl.T @ Xl).astype(np.float64)
    gamma_n = n * 2.0 ** -53 / (1 - n * 2.0 ** -53)
    bound = gamma_n * (np.abs(X.astype(np.float64)).T @ np.abs(X.astype(np.float64)))
    assert np.all(np.abs(G[0] - exact) <= bound)


def test_strided_rows_match_contiguous():
    n, p = 500, 7
    big = workloads.draw_rows(n, 11, 0.0, np.float64, workloads.subseed(901))
    X = big[:, :p]          # row stride 11
    y = np.arange(n, dtype=np.float64)
    a = oracle.gram_folds(X, y, 3, fold_seed=1)
    b = oracle.gram_folds(np.ascontiguousarray(X), y, 3, fold_seed=1)
    for u, v in zip(a, b):
        assert np.array_equal(u, v)


def test_foldid_array_overrides_hash():
    n, p, K = 400, 5, 4
    X = workloads.integer_rows(n, p)
    y = workloads.integer_response(n)
    fid = (np.arange(n) % K).astype(np.uint8)
    G, b, yy, nk = oracle.gram_folds(X, y, K, foldid=fid)
    assert list(nk) == [100] * 4
    Xi = X.astype(np.int64)
    assert np.array_equal(G[1], (Xi[1::4].T @ Xi[1::4]).astype(np.float64))


# ----------------------------------------------------------------- eigen

def test_jacobi_vs_eigvalsh():
    A = workloads.draw_rows(200, 40, 0.6, np.float64, workloads.subseed(902))
    S = A.T @ A / 200
    e = oracle.eigvals(S)
    ref = np.sort(np.linalg.eigvalsh(S))[::-1]
    assert np.max(np.abs(e - ref)) <= 1e-13 * ref[0]


@pytest.mark.parametrize("p", [2, 17, 60])
def test_jacobi_tridiagonal_toeplitz_closed_form(p):
    """Eigenvalues of tridiag(b, a, b) are a + 2 b cos(k pi / (p + 1))."""
    a, b = 1.3, -0.45
    T = a * np.eye(p) + b * (np.eye(p, k=1) + np.eye(p, k=-1))
    closed = np.sort(a + 2 * b * np.cos(np.arange(1, p + 1) * math.pi / (p + 1)))[::-1]
    assert np.max(np.abs(oracle.eigvals(T) - closed)) <= 1e-14 * 4


@pytest.mark.parametrize("p,rho", [(5, 0.25), (50, 0.5), (100, 0.9)])
def test_d_compound_symmetry_closed_form(p, rho):
    """(1 - rho) I + rho 11^T has top eigenvalue 1 + (p - 1) rho."""
    A = (1 - rho) * np.eye(p) + rho * np.ones((p, p))
    lam1 = 1 + (p - 1) * rho
    d = oracle.oem_d(A)
    assert abs(d / (1 + 1e-10) - lam1) <= 1e-13 * lam1
    assert d >= lam1


def test_d_identity_and_diagonal():
    assert oracle.oem_d(np.eye(6)) == pytest.approx(1 + 1e-10, rel=1e-15)
    D = np.diag([0.5, 3.0, 2.0])
    assert oracle.oem_d(D) == pytest.approx(3.0 * (1 + 1e-10), rel=1e-15)


def test_standardize_unit_diagonal():
    X = workloads.draw_rows(1000, 6, 0.3, np.float64, workloads.subseed(903),
                            col_scale=np.array([0.1, 1, 10, 3, 0.5, 2.0]))
    G = X.T @ X / 1000
    c = X.T @ np.ones(1000) / 1000
    Gs, cs, s = oracle.standardize(G, c)
    assert np.allclose(np.diag(Gs), 1.0, rtol=0, atol=1e-15)
    assert np.allclose(s, np.sqrt(np.diag(G)), rtol=1e-15)
    assert np.allclose(Gs, G / np.outer(s, s), rtol=1e-15)
    assert np.allclose(cs, c / s, rtol=1e-15)
