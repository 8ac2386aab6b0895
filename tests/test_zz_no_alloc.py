"""oem_gram_noalloc (the Gram pass that allocates nothing) against oem_gram,
through the C ABI: the same kernels and the same plan, only the workspace
differs, so the per-fold sums must be bit-identical.  Two calls in a row on
the same handle type, the second with a smaller input, so the shared static
workspace is reused with stale contents from the first."""
import numpy as np
import pytest

import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _oem():
    import paper_1801_09661_amd as oem
    return oem


def _sums(oem, X, y, K, prec, seed, noalloc, foldid=None):
    with oem.Gram(X.shape[1], K, prec, X.dtype, seed) as g:
        g.add(X, y, foldid=foldid, noalloc=noalloc)
        torch.cuda.synchronize()
        return [t.cpu().numpy() for t in g.export()]


@pytest.mark.parametrize("prec,K", [("fp64", 1), ("fp64", 5), ("split_bf16", 1),
                                    ("split_bf16", 10), ("bf16", 3)])
def test_noalloc_matches_oem_gram(prec, K):
    oem = _oem()
    print(f"case: noalloc Gram {prec} K={K}", flush=True)
    seed = 555
    for n, p, tag in [(70_001, 37, 400), (20_000, 37, 401)]:      # second call smaller
        pr = workloads.tall_multi(n=n, p=p, seed_tag=tag)
        X = torch.from_numpy(pr.X).cuda()
        y = torch.from_numpy(pr.y).cuda()
        ref = _sums(oem, X, y, K, prec, seed, False)
        got = _sums(oem, X, y, K, prec, seed, True)
        for a, b in zip(got, ref):
            assert np.array_equal(a, b), (prec, K, n)


def test_noalloc_accumulates_blocks_and_rejects_oversize():
    """Two row blocks through the no-alloc pass add up like one oem_gram pass
    over both within the FP64 rounding bound (different split plan), fold ids
    follow the global row index; a pass whose workspace would exceed the
    static limit is refused before any work is enqueued."""
    oem = _oem()
    print("case: noalloc blocks and size limit", flush=True)
    K, seed = 4, 77
    pr = workloads.tall_multi(n=60_000, p=24, seed_tag=402)
    X = torch.from_numpy(pr.X).cuda()
    y = torch.from_numpy(pr.y).cuda()
    ref = _sums(oem, X, y, K, "fp64", seed, False)
    with oem.Gram(24, K, "fp64", X.dtype, seed) as g:
        g.add(X[:35_000], y[:35_000], row_offset=0, noalloc=True)
        g.add(X[35_000:], y[35_000:], row_offset=35_000, noalloc=True)
        got = [t.cpu().numpy() for t in g.export()]
        assert np.array_equal(got[3], ref[3])                       # n_k exact
        X64 = pr.X.astype(np.float64)
        bound = 4 * 60_000 * 2.0 ** -53 * (np.abs(X64).T @ np.abs(X64))
        assert np.all(np.abs(got[0].sum(0) - ref[0].sum(0)) <= bound)
        # 20M rows with 4 folds need 80 MB of row lists: refused before any
        # work is enqueued (real, zero-filled buffers all the same), sums untouched
        big = torch.zeros((20_000_000, 24), dtype=torch.float32, device="cuda")
        ybig = torch.zeros(20_000_000, dtype=torch.float64, device="cuda")
        with pytest.raises(oem.OemError) as e:
            g.add(big, ybig, row_offset=60_000, noalloc=True)
        assert e.value.code == oem.OEM_E_INVAL and "workspace" in str(e.value)
        del big, ybig
        again = [t.cpu().numpy() for t in g.export()]
        for a, b in zip(again, got):
            assert np.array_equal(a, b)
