"""GPU parity of the streaming Gram pass (per-fold X^T X, X^T y, y^T y, n)
against the oracle's row loops."""
import numpy as np
import pytest

import oracle
import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _oem():
    import paper_1801_09661_amd as oem
    return oem


def _gram(X, y, K=1, seed=0, foldid=None, blocks=None, precision="fp64"):
    oem = _oem()
    Xd = torch.from_numpy(np.ascontiguousarray(X)).cuda()
    yd = torch.from_numpy(y).cuda()
    fd = None if foldid is None else torch.from_numpy(foldid).cuda()
    with oem.Gram(X.shape[1], K, precision, Xd.dtype, seed) as g:
        if blocks is None:
            g.add(Xd, yd, foldid=fd)
        else:
            for r0, r1 in blocks:
                g.add(Xd[r0:r1], yd[r0:r1], row_offset=r0,
                      foldid=None if fd is None else fd[r0:r1])
        G, b, yy, nk = g.export()
        torch.cuda.synchronize()
        return G.cpu().numpy(), b.cpu().numpy(), yy.cpu().numpy(), nk.cpu().numpy()


@pytest.mark.parametrize("p", [1, 7, 15, 16, 17, 20, 100, 127, 128, 129, 200])
@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_integer_gram_bit_exact(p, dtype):
    n = 3001
    print(f"case: integer gram n={n} p={p} dtype={dtype.__name__}", flush=True)
    X = workloads.integer_rows(n, p, dtype=dtype)
    y = workloads.integer_response(n)
    G, b, yy, nk = _gram(X, y)
    Go, bo, yyo, nko = oracle.gram_folds(X, y, 1)
    assert np.array_equal(G, Go) and np.array_equal(b, bo)
    assert np.array_equal(yy, yyo) and np.array_equal(nk, nko)


@pytest.mark.parametrize("K,p", [(2, 9), (5, 33), (10, 50), (7, 130)])
def test_fold_hash_gram_bit_exact(K, p):
    n = 20011
    seed = 180109661 + K
    print(f"case: fold gram n={n} p={p} K={K}", flush=True)
    X = workloads.integer_rows(n, p)
    y = workloads.integer_response(n)
    G, b, yy, nk = _gram(X, y, K, seed)
    Go, bo, yyo, nko = oracle.gram_folds(X, y, K, seed)
    assert np.array_equal(nk, nko)             # fold assignment is bit-exact
    assert np.array_equal(G, Go) and np.array_equal(b, bo) and np.array_equal(yy, yyo)
    assert np.array_equal(G.sum(axis=0), oracle.gram_train(X, y, -1)[0])


def test_foldid_array_and_row_blocks():
    n, p, K = 9000, 21, 4
    X = workloads.integer_rows(n, p)
    y = workloads.integer_response(n)
    fid = ((np.arange(n) * 7) % K).astype(np.uint8)
    print("case: foldid array + 3 row blocks", flush=True)
    G, b, yy, nk = _gram(X, y, K, foldid=fid, blocks=[(0, 1000), (1000, 1001), (1001, n)])
    Go, bo, yyo, nko = oracle.gram_folds(X, y, K, foldid=fid)
    assert np.array_equal(G, Go) and np.array_equal(b, bo) and np.array_equal(nk, nko)
    # hashed folds over row blocks keep global row indices
    print("case: hashed folds over row blocks", flush=True)
    G2, _, _, nk2 = _gram(X, y, K, seed=3, blocks=[(0, 4097), (4097, n)])
    Go2, _, _, nko2 = oracle.gram_folds(X, y, K, 3)
    assert np.array_equal(G2, Go2) and np.array_equal(nk2, nko2)


@pytest.mark.parametrize("n,p,rho", [(50_000, 100, 0.5), (30_000, 257, 0.3)])
def test_random_gram_within_rounding_bound(n, p, rho):
    print(f"case: random gram n={n} p={p}", flush=True)
    X = workloads.draw_rows(n, p, rho, np.float32, workloads.subseed(77, p))
    y = workloads.response(X, np.ones(p) / p, 1.0, workloads.subseed(78, p))
    G, b, yy, nk = _gram(X, y)
    Go, bo, yyo, _ = oracle.gram_folds(X, y, 1)
    A = np.abs(X.astype(np.float64))
    gamma_n = 2 * n * 2.0 ** -53
    assert np.all(np.abs(G[0] - Go[0]) <= gamma_n * (A.T @ A))
    assert np.all(np.abs(b[0] - bo[0]) <= gamma_n * (A.T @ np.abs(y)))
    assert abs(yy[0] - yyo[0]) <= gamma_n * yyo[0]
    assert np.array_equal(G[0], G[0].T)


def test_small_n_and_single_row():
    for n in [1, 3, 31, 33]:
        X = workloads.integer_rows(n, 5)
        y = workloads.integer_response(n)
        G, b, yy, nk = _gram(X, y)
        Go, bo, yyo, nko = oracle.gram_folds(X, y, 1)
        assert np.array_equal(G, Go) and np.array_equal(nk, nko)


def test_strided_rows():
    n, p = 2000, 13
    big = workloads.integer_rows(n, 20)
    X = big[:, :p]
    y = workloads.integer_response(n)
    oem = _oem()
    Xd = torch.from_numpy(big).cuda()[:, :p]
    yd = torch.from_numpy(y).cuda()
    with oem.Gram(p, 1) as g:
        g.add(Xd, yd)
        G, b, yy, nk = g.export()
    Go, bo, _, _ = oracle.gram_folds(np.ascontiguousarray(X), y, 1)
    assert np.array_equal(G.cpu().numpy(), Go)


def test_deterministic_repeat():
    n, p = 40_000, 60
    X = workloads.draw_rows(n, p, 0.5, np.float32, workloads.subseed(79))
    y = np.ones(n)
    a = _gram(X, y, 3, 5)
    b = _gram(X, y, 3, 5)
    for u, v in zip(a, b):
        assert np.array_equal(u, v)


# ---------------------------------------------------------------- BF16 forms
# Integer X in [-8, 8] is exact in BF16 (hi = x, lo = 0) and every partial
# sum here stays far below 2^24, so the mixed forms must also be bit-exact.

@pytest.mark.parametrize("precision", ["split_bf16", "bf16"])
@pytest.mark.parametrize("p,K", [(1, 1), (20, 1), (32, 1), (33, 1), (100, 1), (128, 1), (129, 1),
                                 (300, 1), (50, 10), (161, 4)])
def test_integer_gram_bit_exact_bf16(precision, p, K):
    n = 5003
    print(f"case: integer gram {precision} n={n} p={p} K={K}", flush=True)
    X = workloads.integer_rows(n, p)
    y = workloads.integer_response(n)
    G, b, yy, nk = _gram(X, y, K, 17, precision=precision)
    Go, bo, yyo, nko = oracle.gram_folds(X, y, K, 17)
    assert np.array_equal(nk, nko)
    assert np.array_equal(G, Go) and np.array_equal(b, bo) and np.array_equal(yy, yyo)


@pytest.mark.parametrize("precision,bound", [("split_bf16", 2e-6), ("bf16", 2e-2)])
@pytest.mark.parametrize("n,p,rho", [(200_000, 100, 0.5), (60_000, 257, 0.3)])
def test_random_gram_bf16_error(precision, bound, n, p, rho):
    """Entry error relative to sum_i |x_i||x_j|: split-BF16 carries ~2^-16 per
    product plus FP32 accumulation within a row split; single BF16 ~2^-8.
    The diagonal, X^T y and y^T y are FP64 in both forms."""
    print(f"case: random gram {precision} n={n} p={p}", flush=True)
    X = workloads.draw_rows(n, p, rho, np.float32, workloads.subseed(81, p))
    y = workloads.response(X, np.ones(p) / p, 1.0, workloads.subseed(82, p))
    G, b, yy, nk = _gram(X, y, precision=precision)
    Go, bo, yyo, _ = oracle.gram_folds(X, y, 1)
    A = np.abs(X.astype(np.float64))
    scale = A.T @ A
    rel = np.abs(G[0] - Go[0]) / scale
    print(f"  max entry error / sum|x_i x_j| = {rel.max():.3e}")
    assert rel.max() <= bound
    gamma_n = 2 * n * 2.0 ** -53
    assert np.all(np.abs(np.diag(G[0]) - np.diag(Go[0])) <= gamma_n * np.diag(scale))
    assert np.all(np.abs(b[0] - bo[0]) <= gamma_n * (A.T @ np.abs(y)))
    assert abs(yy[0] - yyo[0]) <= gamma_n * yyo[0]
    assert np.array_equal(G[0], G[0].T)
