"""Pins of the oracle's sparse-row Gram (Section 5.8: sparse design
matrices): the per-fold sums from compressed sparse rows equal the sums of
the densified rows (the dense oracle's row loops, and scipy's sparse
products), bit for bit for integer entries."""
import numpy as np
import pytest
from scipy import sparse

import oracle
import workloads


def _dense(sp):
    return sparse.csr_matrix((sp.val, sp.col, sp.rowptr), shape=(len(sp.rowptr) - 1, sp.p)).toarray()


def test_integer_sparse_equals_dense_folds():
    sp = workloads.sparse_rows(n=3000, p=40, density=0.08, seed_tag=90, integer=True)
    K, seed = 3, 5
    Gs, bs, yys, nks = oracle.gram_csr(sp.rowptr, sp.col, sp.val, sp.p, sp.y, K, seed)
    Xd = np.ascontiguousarray(_dense(sp))
    Gd, bd, yyd, nkd = oracle.gram_folds(Xd, sp.y, K, seed)
    assert np.array_equal(Gs, Gd) and np.array_equal(bs, bd)
    assert np.array_equal(yys, yyd) and np.array_equal(nks, nkd)


def test_sparse_equals_scipy_products():
    sp = workloads.sparse_rows(n=5000, p=60, density=0.02, seed_tag=91)
    G, b, yy, nk = oracle.gram_csr(sp.rowptr, sp.col, sp.val, sp.p, sp.y)
    A = sparse.csr_matrix((sp.val, sp.col, sp.rowptr), shape=(5000, 60))
    Gref = (A.T @ A).toarray()
    Ad = np.abs(A).toarray()
    bound = 4 * 2.0 ** -53 * 60 * (Ad.T @ Ad)
    assert np.all(np.abs(G[0] - Gref) <= bound + 1e-300)
    assert np.allclose(b[0], A.T @ sp.y, rtol=1e-12, atol=1e-12)
    assert nk[0] == 5000 and yy[0] == pytest.approx(float(sp.y @ sp.y), rel=1e-14)


def test_repeated_columns_add_and_empty_rows():
    # row 0: columns 2, 2, 5 (the two 2s add); row 1 empty; row 2: column 0
    rowptr = np.array([0, 3, 3, 4])
    col = np.array([2, 2, 5, 0], dtype=np.int32)
    val = np.array([1.0, 2.0, -4.0, 3.0])
    y = np.array([1.0, 2.0, -1.0])
    G, b, yy, nk = oracle.gram_csr(rowptr, col, val, 6, y)
    X = np.zeros((3, 6))
    X[0, 2], X[0, 5], X[2, 0] = 3.0, -4.0, 3.0
    assert np.array_equal(G[0], X.T @ X)
    assert np.array_equal(b[0], X.T @ y)
    assert nk[0] == 3 and yy[0] == 6.0


def test_out_of_range_column_rejected():
    with pytest.raises(ValueError):
        oracle.gram_csr(np.array([0, 1]), np.array([7], dtype=np.int32), np.array([1.0]), 6,
                        np.array([0.0]))
