#!/usr/bin/env python3
"""Benchmark: one step = the whole hot path on the tall multi-penalty workload.

Workload (n = 1,000,000, p = 100): rows N(0, Sigma) with AR(1) Sigma_ij =
0.5^|i-j|, X stored FP32, 10 nonzero coefficients +-U(0.5, 2), unit noise;
penalties lasso, elastic net (alpha 0.5), MCP (gamma 3), SCAD (gamma 3.7);
100 lambdas each from lambda_max down to 1e-3 lambda_max; tol 1e-10.

A step is: reset the statistics, one streaming Gram pass over the 400 MB of X
(already resident in HBM), standardisation, d, lambda grids and the four
warm-started paths.  value = lambda-path fits per second of whole steps
(4 fits per step) in the chosen (mixed: split-BF16 Gram) form; the plain FP64
form is timed the same way and reported beside it.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Gram GB/s of X; λ-path fits/s mixed vs FP64; serve p50/p99 at 1e-6 error"
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6
MFMA_BF16_PEAK_TFLOPS = 2500.0

PENALTIES = [dict(kind="lasso"), dict(kind="enet", alpha=0.5), dict(kind="mcp", gamma=3.0),
             dict(kind="scad", gamma=3.7)]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=1_000_000)
    ap.add_argument("--p", type=int, default=100)
    ap.add_argument("--nlambda", type=int, default=100)
    ap.add_argument("--precision", default="split_bf16", choices=["fp64", "split_bf16", "bf16"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-rows", type=int, default=100_000)
    ap.add_argument("--profile-steps", type=int, default=0,
                    help="run only this many steps (for profilers) and skip the baseline")
    ap.add_argument("--serve", action="store_true",
                    help="serving workload instead: Poisson arrivals of fit / CV requests")
    ap.add_argument("--requests", type=int, default=2000)
    ap.add_argument("--rate", type=float, default=50.0)
    ap.add_argument("--slots", type=int, default=8)
    ap.add_argument("--batch", action="store_true",
                    help="batched uneven workload instead (64 problems, p log-uniform in [16, 2048], n = 200 p)")
    ap.add_argument("--cv", action="store_true",
                    help="grouped 10-fold CV workload instead (n=2e6, p=500, group lasso + lasso + MCP)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="after the steps, copy X once with a plain device copy (traffic calibration)")
    return ap.parse_args()


# HBM traffic per launch from rocprofv3 FETCH_SIZE / WRITE_SIZE passes, kept
# in profiles/ with the hash of the kernel sources they were taken on; a
# changed source makes the stored figures stale and traffic is reported null.
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_tall_multi.txt")
TRAFFIC_SOURCES = {"gram": ["gram_bf16.hip", "gram_common.hip", "gram_common.h"],
                   "fit": ["derive.hip", "path.hip", "path_reg.hip", "path_stream.hip", "path_ws.hip",
                           "path_common.h"]}


def sources_hash(phase):
    import hashlib
    h = hashlib.sha256()
    for name in TRAFFIC_SOURCES[phase]:
        with open(os.path.join(ROOT, "paper_1801_09661_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def stored_traffic():
    """{phase: bytes per launch} from the traffic summary; a phase whose
    kernel sources changed since the counters were taken is left out."""
    if not os.path.exists(TRAFFIC_FILE):
        return {}
    vals, digest = {}, {}
    with open(TRAFFIC_FILE) as f:
        for line in f:
            parts = line.split()
            if len(parts) == 3 and parts[0] == "sources_sha256":
                digest[parts[1]] = parts[2]
            elif len(parts) == 3 and parts[0] == "traffic_bytes":
                vals[parts[1]] = float(parts[2])
    return {k: v for k, v in vals.items() if k in TRAFFIC_SOURCES and digest.get(k) == sources_hash(k)}


def cpu_baseline(pr, nlambda, sample_rows):
    """Oracle (single-threaded plain C, FP64) on a bounded sample: the Gram
    pass on the first `sample_rows` rows, scaled linearly to n, plus the four
    paths on that sample's statistics (path work does not depend on n)."""
    import numpy as np
    import oracle
    n = pr.X.shape[0]
    Xs = np.ascontiguousarray(pr.X[:sample_rows])
    ys = pr.y[:sample_rows]
    t0 = time.perf_counter()
    G, b, yy, ns = oracle.gram_train(Xs, ys, -1)
    t_gram = time.perf_counter() - t0
    t0 = time.perf_counter()
    st = oracle.prepare(G, b, yy, ns, True)
    lam = oracle.lambda_sequences(st["cs"], PENALTIES, nlambda, 1e-3)
    oracle.fit_from_stats(st, PENALTIES, lam, tol=1e-10)
    t_path = time.perf_counter() - t0
    t_full = t_gram * (n / sample_rows) + t_path
    return dict(value=len(PENALTIES) / t_full, unit="fits/s", cores=1, kind="oracle",
                sample=f"Gram on {sample_rows} of {n} rows ({t_gram:.2f} s, scaled x{n / sample_rows:.0f}) "
                       f"+ 4 paths x {nlambda} lambdas on the sample's statistics ({t_path:.2f} s)",
                seconds_per_step=t_full)


def run_form(oem, torch, X, y, precision, steps, warm, nlambda):
    """Time `steps` whole steps of one precision form; then phase split."""
    import numpy as np
    n, p = X.shape
    g = oem.Gram(p, 1, precision, X.dtype)
    stream = torch.cuda.current_stream()
    ev = lambda: torch.cuda.Event(enable_timing=True)

    def step(record=None):
        oem.oem_gram_reset(g.h)
        if record is not None:
            record[0].record(stream)
        g.add(X, y)
        if record is not None:
            record[1].record(stream)
        res = g.fit_path(PENALTIES, nlambda=nlambda, lambda_min_ratio=1e-3, tol=1e-10,
                         maxit=100000, sync=False)
        if record is not None:
            record[2].record(stream)
        return res

    for _ in range(warm):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        res = step()
    torch.cuda.synchronize()
    t_steps = time.perf_counter() - t0

    gram_ms, fit_ms = [], []
    for _ in range(3):
        rec = [ev(), ev(), ev()]
        res = step(rec)
        torch.cuda.synchronize()
        gram_ms.append(rec[0].elapsed_time(rec[1]))
        fit_ms.append(rec[1].elapsed_time(rec[2]))
    # Gram pass alone, back to back: average launch duration of the pass
    reps = 20
    a, b = ev(), ev()
    a.record(stream)
    for _ in range(reps):
        g.add(X, y)
    b.record(stream)
    torch.cuda.synchronize()
    gram_only_ms = a.elapsed_time(b) / reps
    iters = res["iters"].cpu().numpy()
    beta = res["beta"].cpu().numpy()
    g.close()
    return dict(t_steps=t_steps, ms_per_step=1e3 * t_steps / steps,
                fits_per_s=len(PENALTIES) * steps / t_steps, gram_ms=float(np.mean(gram_ms)),
                fit_ms=float(np.mean(fit_ms)), gram_only_ms=gram_only_ms,
                updates=int(np.abs(iters).sum()), beta=beta)


CV_PENALTIES = [dict(kind="grp_lasso"), dict(kind="lasso"), dict(kind="mcp", gamma=3.0)]


def cv_main(args):
    """Grouped 10-fold CV workload: n = 2e6, p = 500, AR(1) rho = 0.3 FP32 X,
    50 contiguous groups of 10 (5 active), sigma = 2; group lasso, lasso and
    MCP (gamma 3), 100 lambdas.  A step is one Gram pass with fold sums
    followed by oem_cv (10 folds + the full data = 33 paths, CV error and
    selection), timed for the split-BF16 and the FP64 forms."""
    import numpy as np
    import torch
    import paper_1801_09661_amd as oem
    import workloads

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    oem.load_library()
    n = 2_000_000 if args.n == 1_000_000 else args.n
    p = 500 if args.p == 100 else args.p
    K = 10
    pr = workloads.cv_grouped(n=n, p=p)
    X = torch.from_numpy(pr.X).cuda()
    y = torch.from_numpy(pr.y).cuda()
    groups = pr.groups
    del pr
    torch.cuda.synchronize()
    steps = args.profile_steps or args.steps
    warm = 0 if args.profile_steps else args.warmup
    forms = [args.precision] if args.profile_steps else [args.precision, "fp64"]
    if args.precision == "fp64":
        forms = ["fp64"]
    stream = torch.cuda.current_stream()
    ev = lambda: torch.cuda.Event(enable_timing=True)
    runs = {}
    for form in forms:
        g = oem.Gram(p, K, form, X.dtype, 180109661)
        # the library's Gram autotuner picks the workgroup count for this
        # shape once, untimed (it leaves the sums cleared); both forms are tuned
        oem.oem_gram_autotune(g.h, X, y)

        def step(rec=None):
            oem.oem_gram_reset(g.h)
            if rec is not None:
                rec[0].record(stream)
            g.add(X, y)
            if rec is not None:
                rec[1].record(stream)
            r = g.cv(CV_PENALTIES, nlambda=args.nlambda, lambda_min_ratio=1e-3, tol=1e-10,
                     groups=groups, sync=False)
            if rec is not None:
                rec[2].record(stream)
            return r

        for _ in range(warm):
            step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            res = step()
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        rec = [ev(), ev(), ev()]
        res = step(rec)
        torch.cuda.synchronize()
        runs[form] = dict(ms_per_step=1e3 * t / steps, fits_per_s=(K + 1) * len(CV_PENALTIES) * steps / t,
                          gram_ms=rec[0].elapsed_time(rec[1]), cv_ms=rec[1].elapsed_time(rec[2]),
                          updates=int(np.abs(res["iters"].cpu().numpy()).sum()),
                          beta=res["beta"].cpu().numpy())
        g.close()
    main_run = runs[args.precision]
    x_bytes = n * p * X.element_size() + n * 8
    out = {
        "metric": METRIC,
        "value": main_run["fits_per_s"],
        "unit": "fits/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warm,
        "ms_per_step": main_run["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp64": "f64", "split_bf16": "split-bf16 Gram (f32 acc, f64 reduce) + f64 paths",
                  "bf16": "bf16 Gram (f32 acc, f64 reduce) + f64 paths"}[args.precision],
        "data": "synthetic",
        "config": {"workload": "cv_grouped: n=2e6 p=500 AR(1) rho=0.3 FP32 X, 10 hashed folds, 50 groups "
                               "of 10 (5 active), group lasso+lasso+MCP, 100 lambdas, tol 1e-10",
                   "n": n, "p": p, "folds": K, "penalties": len(CV_PENALTIES), "nlambda": args.nlambda,
                   "precision": args.precision},
        "gram_ms_in_step": main_run["gram_ms"],
        "cv_ms_in_step": main_run["cv_ms"],
        "gram_gbps": x_bytes / (main_run["gram_ms"] * 1e-3) / 1e9,
        "oem_updates": main_run["updates"],
    }
    if "fp64" in runs and args.precision != "fp64":
        f64 = runs["fp64"]
        out["fp64_form"] = dict(fits_per_s=f64["fits_per_s"], ms_per_step=f64["ms_per_step"],
                                gram_ms_in_step=f64["gram_ms"], cv_ms_in_step=f64["cv_ms"])
        out["mixed_vs_fp64_fits"] = main_run["fits_per_s"] / f64["fits_per_s"]
        bm, bf = main_run["beta"], f64["beta"]
        scale = np.maximum(np.abs(bf).max(axis=2), 1e-300)
        out["mixed_coef_err_vs_fp64_form"] = float((np.abs(bm - bf).max(axis=2) / scale)[:, 1:].max())
    print(json.dumps(out))


def batch_main(args):
    """Batched uneven workload: 64 independent problems, p log-uniform in
    [16, 2048], n = 200 p, FP32 N(0,1) columns with log-uniform scales in
    [0.1, 10], 5% nonzero coefficients; lasso, 100 lambdas.  A step is one
    replay of the batch's captured hipGraph (Gram passes, d, paths of every
    problem), for the split-BF16 and the FP64 forms; the per-problem
    coefficient error of the mixed form against the FP64 form is reported."""
    import numpy as np
    import torch
    import paper_1801_09661_amd as oem
    import workloads

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    oem.load_library()
    shapes = workloads.batched_uneven_shapes(64)
    dev = []
    for i, (n, p) in enumerate(shapes):
        pr = workloads.batched_uneven_problem(i, n, p)
        dev.append((torch.from_numpy(pr.X).cuda(), torch.from_numpy(pr.y).cuda()))
        del pr
    torch.cuda.synchronize()
    steps = args.profile_steps or args.steps
    warm = 0 if args.profile_steps else args.warmup
    forms = [args.precision] if args.profile_steps else [args.precision, "fp64"]
    if args.precision == "fp64":
        forms = ["fp64"]
    s = torch.cuda.Stream()
    runs = {}
    for form in forms:
        with oem.Batch(dev, ["lasso"], precision=form, nlambda=args.nlambda, tol=1e-10) as b:
            with torch.cuda.stream(s):
                for _ in range(max(warm, 1)):
                    b.run(graph=True, stream=s)
            s.synchronize()
            t0 = time.perf_counter()
            with torch.cuda.stream(s):
                for _ in range(steps):
                    b.run(graph=True, stream=s)
            s.synchronize()
            t = time.perf_counter() - t0
            assert b.status(stream=s) == oem.OEM_OK
            runs[form] = dict(ms_per_step=1e3 * t / steps, fits_per_s=len(dev) * steps / t,
                              beta=[o["beta"].cpu().numpy() for o in b.out],
                              updates=int(sum(np.abs(o["iters"].cpu().numpy()).sum() for o in b.out)))
    main_run = runs[args.precision]
    out = {
        "metric": METRIC,
        "value": main_run["fits_per_s"],
        "unit": "fits/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warm,
        "ms_per_step": main_run["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp64": "f64", "split_bf16": "split-bf16 Gram (f32 acc, f64 reduce) + f64 paths",
                  "bf16": "bf16 Gram (f32 acc, f64 reduce) + f64 paths"}[args.precision],
        "data": "synthetic",
        "config": {"workload": "batched_uneven: 64 problems, p log-uniform in [16,2048], n=200p, FP32 X with "
                               "column scales in [0.1,10], lasso, 100 lambdas, one hipGraph replay per step",
                   "problems": len(dev), "p_max": max(p for _, p in shapes), "nlambda": args.nlambda,
                   "precision": args.precision},
        "oem_updates": main_run["updates"],
    }
    if "fp64" in runs and args.precision != "fp64":
        f64 = runs["fp64"]
        out["fp64_form"] = dict(fits_per_s=f64["fits_per_s"], ms_per_step=f64["ms_per_step"])
        out["mixed_vs_fp64_fits"] = main_run["fits_per_s"] / f64["fits_per_s"]
        errs = []
        for bm, bf in zip(main_run["beta"], f64["beta"]):
            scale = np.maximum(np.abs(bf).max(axis=2), 1e-300)
            errs.append(float((np.abs(bm - bf).max(axis=2) / scale)[:, 1:].max()))
        out["mixed_coef_err_vs_fp64_form_max"] = max(errs)
        out["mixed_coef_err_vs_fp64_form_median"] = float(np.median(errs))
    print(json.dumps(out))


def serve_main(args):
    """Serving workload: requests with Poisson arrivals at `rate`/s, p
    log-uniform in [10, 1000], n log-uniform in [1e4, 1e6] (n >= 10 p),
    AR(1) rows in pinned host memory, penalty uniform over lasso / MCP / SCAD
    / group lasso (groups of 5), 20% with 5-fold CV, 100 lambdas, split-BF16
    Gram.  Latency runs from arrival to the result in host memory.  Prints
    one JSON line."""
    import numpy as np
    import torch
    from concurrent.futures import ThreadPoolExecutor
    import paper_1801_09661_amd as oem
    import workloads
    import oracle

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    oem.load_library()
    reqs = workloads.serving_requests(count=args.requests, rate_per_s=args.rate)
    nmax, pmax = max(r.n for r in reqs), max(r.p for r in reqs)
    t0 = time.perf_counter()
    pool = {}
    for bk in sorted({workloads.serving_bucket(r.rho) for r in reqs}):
        pool[bk] = torch.from_numpy(workloads.serving_pool(nmax, pmax, bk)).pin_memory()
    views = [pool[workloads.serving_bucket(r.rho)][:r.n, :r.p] for r in reqs]
    offs = np.concatenate([[0], np.cumsum([r.n for r in reqs])])
    yall = torch.empty(int(offs[-1]), dtype=torch.float64).pin_memory()

    def make_y(i):
        y, _ = workloads.serving_response(reqs[i], views[i].numpy())
        yall[int(offs[i]):int(offs[i + 1])] = torch.from_numpy(y)

    with ThreadPoolExecutor(16) as ex:
        list(ex.map(make_y, range(len(reqs))))
    t_setup = time.perf_counter() - t0
    L = 100
    kinds = {"lasso": "lasso", "mcp": dict(kind="mcp", gamma=3.0), "scad": dict(kind="scad", gamma=3.7),
             "grp_lasso": "grp_lasso"}
    srv = oem.Server(nslots=args.slots, device_bytes=200 << 30, precision="split_bf16", nlambda=L, tol=1e-10)
    start = srv.now() + 0.5
    done = []
    for r, X in zip(reqs, views):
        while srv.now() < start + r.arrival_s:
            done.extend(srv.poll(wait=False))
            time.sleep(0.0005)
        groups = (np.arange(r.p) // 5).astype(np.int32) if r.penalty == "grp_lasso" else None
        srv.submit(r.index, X, yall[int(offs[r.index]):int(offs[r.index + 1])], kinds[r.penalty],
                   nfolds=r.nfolds, fold_seed=r.fold_seed, groups=groups, t_arrival=start + r.arrival_s)
    done.extend(srv.drain())
    srv.close()
    lat = np.array([d["t_done"] - d["t_arrival"] for d in done])
    dev = np.array([d["t_done"] - d["t_admit"] for d in done])
    span = max(d["t_done"] for d in done) - start
    xbytes = sum(r.n * r.p * 4 for r in reqs)
    # accuracy on a sample of small plain fits against the FP64 oracle on the
    # lambdas the request used (untimed)
    res = {d["id"]: d for d in done}
    sample = [r for r in reqs if r.nfolds == 1 and r.p <= 120 and r.n <= 60000][:8]
    worst = 0.0
    for r in sample:
        X = np.ascontiguousarray(views[r.index].numpy())
        y = yall[int(offs[r.index]):int(offs[r.index + 1])].numpy()
        groups = (np.arange(r.p) // 5).astype(np.int32) if r.penalty == "grp_lasso" else None
        ref = oracle.fit(X, y, [kinds[r.penalty]], groups=groups, lambdas=res[r.index]["lambda_"][None, :],
                         tol=1e-10)
        for l in range(1, L):
            sc = np.abs(ref["beta"][0, l]).max()
            if sc > 0:
                worst = max(worst, float(np.abs(res[r.index]["beta"][l] - ref["beta"][0, l]).max() / sc))
    out = {
        "metric": "serve p50/p99 latency (arrival to result in host memory)",
        "value": len(done) / span, "unit": "requests/s", "n_gpus": 1, "higher_is_better": True,
        "p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3),
        "device_p50_ms": float(np.percentile(dev, 50) * 1e3), "device_p99_ms": float(np.percentile(dev, 99) * 1e3),
        "x_gb_per_s": xbytes / span / 1e9, "requests": len(done),
        "not_ok": int(sum(d["status"] != 0 for d in done)), "setup_s": t_setup,
        "coef_err_vs_fp64_oracle_sample": worst, "sample": len(sample),
        "dtype": "split-bf16 Gram (f32 acc, f64 reduce) + f64 paths", "data": "synthetic",
        "config": {"workload": f"serving: {args.requests} requests, Poisson {args.rate}/s, p in [10,1000], "
                               "n in [1e4,1e6], AR(1) rho~U(0,0.8) (8 levels), lasso/MCP/SCAD/group lasso, "
                               "20% 5-fold CV, 100 lambdas", "slots": args.slots},
    }
    print(json.dumps(out))


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    if args.serve:
        return serve_main(args)
    if args.cv:
        return cv_main(args)
    if args.batch:
        return batch_main(args)
    import numpy as np
    import torch
    import paper_1801_09661_amd as oem
    import workloads

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    oem.load_library()
    pr = workloads.tall_multi(n=args.n, p=args.p)
    X = torch.from_numpy(pr.X).cuda()
    y = torch.from_numpy(pr.y).cuda()
    n, p = X.shape
    torch.cuda.synchronize()

    steps = args.profile_steps or args.steps
    warm = 0 if args.profile_steps else args.warmup
    forms = [args.precision] if args.profile_steps else [args.precision, "fp64"]
    if args.precision == "fp64" and not args.profile_steps:
        forms = ["fp64"]
    runs = {f: run_form(oem, torch, X, y, f, steps, warm, args.nlambda) for f in forms}
    main_run = runs[args.precision]

    if args.calibrate_copy:
        Z = torch.empty_like(X)
        Z.copy_(X)
        torch.cuda.synchronize()
        del Z
    traffic = stored_traffic() if args.precision == "split_bf16" else {}
    x_bytes = n * p * X.element_size() + n * 8   # X and y, read once
    gram_gbs = x_bytes / (main_run["gram_only_ms"] * 1e-3) / 1e9
    path_flops = 2.0 * p * p * main_run["updates"]
    path_tflops = path_flops / (main_run["fit_ms"] * 1e-3) / 1e12
    gram_roof = dict(bound="hbm", kernel="gram pass (gram kernel + fixed-order reduction)",
                     achieved=gram_gbs, peak=HBM_PEAK_GBS, unit="GB/s", frac=gram_gbs / HBM_PEAK_GBS,
                     traffic=traffic.get("gram"), algorithmic=f"{x_bytes} B of X and y per launch")
    path_roof = dict(bound="alu", kernel="path kernel (+ combine, Lanczos d, lambda grid)",
                     achieved=path_tflops, peak=FP64_PEAK_TFLOPS, unit="TFLOP/s",
                     frac=path_tflops / FP64_PEAK_TFLOPS, traffic=traffic.get("fit"),
                     algorithmic=f"2 p^2 flops x {main_run['updates']} OEM updates per launch")
    dominant = gram_roof if main_run["gram_ms"] >= main_run["fit_ms"] else path_roof
    out = {
        "metric": METRIC,
        "value": main_run["fits_per_s"],
        "unit": "fits/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warm,
        "ms_per_step": main_run["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp64": "f64", "split_bf16": "split-bf16 Gram (f32 acc, f64 reduce) + f64 paths",
                  "bf16": "bf16 Gram (f32 acc, f64 reduce) + f64 paths"}[args.precision],
        "data": "synthetic",
        "config": {"workload": "tall_multi: n=1e6 p=100 AR(1) rho=0.5 FP32 X, lasso+enet+MCP+SCAD, "
                               "100 lambdas each, tol 1e-10", "n": n, "p": p, "penalties": 4,
                   "nlambda": args.nlambda, "precision": args.precision},
        "gram_ms_in_step": main_run["gram_ms"],
        "fit_ms_in_step": main_run["fit_ms"],
        "gram_gbps": gram_gbs,
        "oem_updates": main_run["updates"],
        "roofline": dominant,
        "gram_roofline": gram_roof,
    }
    if "fp64" in runs and args.precision != "fp64":
        f64 = runs["fp64"]
        out["fp64_form"] = dict(fits_per_s=f64["fits_per_s"], ms_per_step=f64["ms_per_step"],
                                gram_gbps=x_bytes / (f64["gram_only_ms"] * 1e-3) / 1e9,
                                gram_ms_in_step=f64["gram_ms"], fit_ms_in_step=f64["fit_ms"])
        out["mixed_vs_fp64_fits"] = main_run["fits_per_s"] / f64["fits_per_s"]
        bm, bf = main_run["beta"], f64["beta"]
        scale = np.maximum(np.abs(bf).max(axis=2), 1e-300)
        out["mixed_coef_err_vs_fp64_form"] = float((np.abs(bm - bf).max(axis=2) / scale)[:, 1:].max())
    if not args.no_cpu_baseline and not args.profile_steps:
        out["cpu_baseline"] = cpu_baseline(pr, args.nlambda, min(args.cpu_sample_rows, n))
    print(json.dumps(out))


if __name__ == "__main__":
    main()
