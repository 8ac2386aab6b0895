"""GPU sparse-row Gram pass (oem_gram_csr; Section 5.8: sparse design
matrices) through the C ABI.

The kernel densifies each row block in registers and LDS and runs the same
matrix-core tiles as the dense pass, so its sums must equal oem_gram's on
the densified rows bit for bit; against the oracle's sparse row loops they
agree within the FP64 rounding bound, exactly for integer entries; paths on
the paper's sparse example (n = 1e5, p = 200, 1% density, lasso and group
lasso with groups of 5) match the oracle within 1e-10."""
import numpy as np
import pytest
from scipy import sparse

import oracle
import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _oem():
    import paper_1801_09661_amd as oem
    return oem


def _cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _dense(sp, n):
    return np.ascontiguousarray(
        sparse.csr_matrix((sp.val, sp.col, sp.rowptr), shape=(n, sp.p)).toarray())


def _sums(g):
    torch.cuda.synchronize()
    return [t.cpu().numpy() for t in g.export()] + [t.cpu().numpy() for t in g.export_colsums()]


@pytest.mark.parametrize("n,p,density,K,dt", [(30_001, 37, 0.05, 1, np.float64),
                                               (30_001, 37, 0.05, 4, np.float32),
                                               (12_345, 150, 0.02, 3, np.float64),
                                               (8_000, 300, 0.3, 1, np.float32)])
def test_csr_equals_dense_pass(n, p, density, K, dt):
    oem = _oem()
    print(f"case: csr vs dense n={n} p={p} density={density} K={K} {dt.__name__}", flush=True)
    sp = workloads.sparse_rows(n=n, p=p, density=density, seed_tag=700 + p, dtype=dt)
    tdt = torch.float64 if dt == np.float64 else torch.float32
    with oem.Gram(p, K, "fp64", tdt, 11) as g:
        g.add_csr(_cuda(sp.rowptr), _cuda(sp.col), _cuda(sp.val), _cuda(sp.y))
        got = _sums(g)
    with oem.Gram(p, K, "fp64", tdt, 11) as g:
        g.add(_cuda(_dense(sp, n).astype(dt)), _cuda(sp.y))
        ref = _sums(g)
    for a, b in zip(got, ref):
        assert np.array_equal(a, b)


def test_csr_integer_exact_against_oracle_and_bad_columns():
    """Integer entries: sums equal the oracle's sparse row loops bit for bit.
    Entries at columns outside [0, p) are ignored by the kernel."""
    oem = _oem()
    print("case: csr integer exact n=40000 p=64", flush=True)
    n, p, K, seed = 40_000, 64, 5, 3
    sp = workloads.sparse_rows(n=n, p=p, density=0.05, seed_tag=710, integer=True)
    G, b, yy, nk = oracle.gram_csr(sp.rowptr, sp.col, sp.val, p, sp.y, K, seed)
    with oem.Gram(p, K, "fp64", torch.float64, seed) as g:
        g.add_csr(_cuda(sp.rowptr), _cuda(sp.col), _cuda(sp.val), _cuda(sp.y))
        got = _sums(g)
    assert np.array_equal(got[0], G) and np.array_equal(got[1], b)
    assert np.array_equal(got[2], yy) and np.array_equal(got[3], nk)
    # the same rows with an extra entry at column p + 5 and one at -1 in row 0
    rp = sp.rowptr.copy()
    rp[1:] += 2
    col = np.r_[np.array([p + 5, -1], dtype=np.int32), sp.col]
    val = np.r_[np.array([9.0, 9.0]), sp.val]
    with oem.Gram(p, K, "fp64", torch.float64, seed) as g:
        g.add_csr(_cuda(rp), _cuda(col), _cuda(val), _cuda(sp.y))
        bad = _sums(g)
    assert np.array_equal(bad[0], G) and np.array_equal(bad[1], b)


def test_paper_sparse_example_paths():
    """n = 1e5, p = 200, density 1%: lasso and group lasso (groups of 5)
    from the CSR Gram against the oracle's paths on the oracle's sparse sums."""
    oem = _oem()
    print("case: paper sparse example n=1e5 p=200", flush=True)
    sp = workloads.sparse_rows()
    n, p = len(sp.rowptr) - 1, sp.p
    groups = (np.arange(p) // 5).astype(np.int32)
    pens = ["lasso", "grp_lasso"]
    G, b, yy, nk = oracle.gram_csr(sp.rowptr, sp.col, sp.val, p, sp.y)
    st = oracle.prepare(G[0], b[0], yy[0], nk[0])
    lam = oracle.lambda_sequences(st["cs"], pens, 30, 1e-2, groups=groups)
    ref = oracle.fit_from_stats(st, pens, lam, groups=groups, tol=1e-10)
    with oem.Gram(p, 1, "fp64", torch.float64) as g:
        g.add_csr(_cuda(sp.rowptr), _cuda(sp.col), _cuda(sp.val), _cuda(sp.y))
        res = g.fit_path(pens, nlambda=30, lambdas=lam, tol=1e-10, groups=groups)
        torch.cuda.synchronize()
        beta = res["beta"].cpu().numpy()
    for q in range(2):
        for l in range(1, 30):
            s = np.abs(ref["beta"][q, l]).max()
            assert np.abs(beta[q, l] - ref["beta"][q, l]).max() <= 1e-10 * s, (q, l)
            assert np.array_equal(beta[q, l] != 0, ref["beta"][q, l] != 0), (q, l)
