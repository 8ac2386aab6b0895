"""GPU test: several handles, each on its own stream, running whole CV steps
(Gram pass with fold sums + oem_cv) one after another without waiting for
each other, as a caller that keeps several problems in flight does (also
with each next Gram pass enqueued before the current oem_cv).

Each oem_cv waits for its own d, so one multi-workgroup d launch runs at a
time, beside the paths of the steps before it.  Every step runs the same
kernels on the same inputs as the one-handle run, so its outputs must be
bit-identical to it; the one-handle run is checked against the oracle's
held-out error."""
import numpy as np
import pytest

import oracle
import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-10
K = 5
SEED = 4242


def _oem():
    import paper_1801_09661_amd as oem
    return oem


@pytest.mark.parametrize("in_flight,precision,early", [(2, "fp64", False), (3, "fp64", True),
                                                       (3, "split_bf16", True)])
def test_cv_steps_in_flight_match_one_handle(in_flight, precision, early):
    oem = _oem()
    # p > 128: d from the multi-workgroup Lanczos
    pr = workloads.cv_grouped(n=60_000, p=200, group_size=10, active_groups=4, seed_tag=77)
    n, p = pr.X.shape
    X = torch.from_numpy(pr.X).cuda()
    y = torch.from_numpy(pr.y).cuda()
    pens = ["grp_lasso", "lasso", dict(kind="mcp", gamma=3.0)]
    kw = dict(nlambda=30, lambda_min_ratio=1e-2, tol=TOL, groups=pr.groups, sync=False)
    print(f"case: n={n} p={p} K={K}, {precision}, {in_flight} handles in flight, early Gram {early}", flush=True)

    ref_h = oem.Gram(p, K, precision, X.dtype, SEED)
    ref_h.add(X, y)
    ref = ref_h.cv(pens, **kw)
    torch.cuda.synchronize()
    ref_beta = ref["beta"].cpu().numpy()
    ref_cvm = ref["cvm"].cpu().numpy()
    ref_h.close()

    handles = [oem.Gram(p, K, precision, X.dtype, SEED) for _ in range(in_flight)]
    streams = [torch.cuda.Stream() for _ in range(in_flight)]
    def gram_step(i):
        h, st = handles[i % in_flight], streams[i % in_flight]
        with torch.cuda.stream(st):
            oem.oem_gram_reset(h.h, stream=st)
            h.add(X, y, stream=st)

    def cv_step(i):
        h, st = handles[i % in_flight], streams[i % in_flight]
        with torch.cuda.stream(st):
            return h.cv(pens, stream=st, **kw)

    outs = []
    steps = 3 * in_flight
    if early:
        # the next step's Gram pass enqueued before this step's oem_cv: it
        # runs beside this step's d
        gram_step(0)
        for i in range(steps):
            if i + 1 < steps:
                gram_step(i + 1)
            outs.append(cv_step(i))
    else:
        for i in range(steps):
            gram_step(i)
            outs.append(cv_step(i))
    torch.cuda.synchronize()
    for i, r in enumerate(outs):
        assert np.array_equal(r["beta"].cpu().numpy(), ref_beta), f"step {i} beta"
        assert np.array_equal(r["cvm"].cpu().numpy(), ref_cvm), f"step {i} cvm"
    for h in handles:
        h.close()

    if precision != "fp64":
        return   # the mixed forms' error against the oracle is tested with the single fits
    # the one-handle run against the oracle's held-out error (group lasso)
    ref_o = oracle.cv(pr.X, pr.y, K, SEED, ["grp_lasso"], groups=pr.groups, nlambda=30,
                      lambda_min_ratio=1e-2, tol=TOL)
    assert np.allclose(ref_cvm[0], ref_o["cvm"][0], rtol=1e-9, atol=0)
