#!/usr/bin/env python3
"""Benchmark of the OEM hot path on one MI355X.  Prints one JSON line.

Default line: the grouped 10-fold CV workload (n = 2e6, p = 500, AR(1)
rho = 0.3, X stored FP32 (4 GB, resident in HBM), 50 contiguous groups of 10
with 5 active, sigma = 2; group lasso, lasso and MCP gamma = 3; 100 lambdas,
tol 1e-10).  A step is the whole hot path: reset, one Gram pass with the
fold sums, then oem_cv (standardisation and d of the 11 problems, the 33
warm-started paths, CV error and selection).  value = lambda-path fits per
second of whole steps in the mixed form (split-BF16 Gram, FP64 after it);
the plain FP64 form is timed the same way beside it.  Sub-records: the
tall multi-penalty workload (n = 1e6, p = 100), the group MCP / group SCAD /
sparse group lasso paths, the out-of-core pass from host memory, the sparse
example and logistic regression.  Coefficient and objective errors are
against the FP64 oracle's path pipeline.  cpu_baseline times the oracle on
this host, single-threaded and on all cores.

Other lines: --tall (the tall multi-penalty workload as the main line),
--batch (64 uneven problems), --serve (the request loop).
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time
from concurrent.futures import ThreadPoolExecutor

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Gram GB/s of X; λ-path fits/s mixed vs FP64; serve p50/p99 at 1e-6 error"
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6
MFMA_BF16_PEAK_TFLOPS = 2500.0
# CV steps in flight in the default line (--in-flight): each step's oem_cv
# waits for its d, so the host enqueues a step's Gram pass only once the
# previous step's d is in; a fourth step in flight measured no faster than
# three
CV_IN_FLIGHT = 3
DTYPE = {"fp64": "f64", "split_bf16": "split-bf16 Gram (f32 acc, f64 reduce) + f64 paths",
         "bf16": "bf16 Gram (f32 acc, f64 reduce) + f64 paths"}

TALL_PENALTIES = [dict(kind="lasso"), dict(kind="enet", alpha=0.5), dict(kind="mcp", gamma=3.0),
                  dict(kind="scad", gamma=3.7)]
CV_PENALTIES = [dict(kind="grp_lasso"), dict(kind="lasso"), dict(kind="mcp", gamma=3.0)]
GROUP_PENALTIES = [dict(kind="grp_mcp", gamma=3.0), dict(kind="grp_scad", gamma=3.7),
                   dict(kind="sgl", tau=0.5)]
CV_SEED = 180109661


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--in-flight", type=int, default=CV_IN_FLIGHT,
                    help="CV line: problems in flight on as many streams and handles")
    ap.add_argument("--n", type=int, default=0, help="rows (default: the workload's)")
    ap.add_argument("--p", type=int, default=0, help="columns (default: the workload's)")
    ap.add_argument("--nlambda", type=int, default=100)
    ap.add_argument("--precision", default="split_bf16", choices=["fp64", "split_bf16", "bf16"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--sequential", action="store_true",
                    help="CV line: one problem in flight (default: three, on three streams)")
    ap.add_argument("--no-extras", action="store_true", help="skip the sub-records and the oracle errors")
    ap.add_argument("--profile-steps", type=int, default=0,
                    help="run only this many steps of the main form (for profilers); no extras")
    ap.add_argument("--cv", action="store_true", help="grouped 10-fold CV workload (the default)")
    ap.add_argument("--tall", action="store_true", help="tall multi-penalty workload as the main line")
    ap.add_argument("--serve", action="store_true",
                    help="serving workload instead: Poisson arrivals of fit / CV requests")
    ap.add_argument("--requests", type=int, default=2000)
    ap.add_argument("--rate", type=float, default=50.0)
    ap.add_argument("--slots", type=int, default=8)
    ap.add_argument("--batch", action="store_true",
                    help="batched uneven workload instead (64 problems, p log-uniform in [16, 2048], n = 200 p)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="after the steps, copy X once with a plain device copy (traffic calibration)")
    return ap.parse_args()


# HBM traffic per launch from rocprofv3 FETCH_SIZE / WRITE_SIZE passes, kept
# in profiles/ with the hash of the kernel sources they were taken on; a
# changed source makes the stored figures stale and traffic is reported null.
TRAFFIC_SOURCES = {"gram": ["gram_bf16.hip", "gram.hip", "gram_common.hip", "gram_common.h"]}


def sources_hash(phase):
    import hashlib
    h = hashlib.sha256()
    for name in TRAFFIC_SOURCES[phase]:
        with open(os.path.join(ROOT, "paper_1801_09661_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def stored_traffic(workload):
    """{phase: bytes per launch} from profiles/traffic_<workload>.txt; a phase
    whose kernel sources changed since the counters were taken is left out."""
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}.txt")
    if not os.path.exists(path):
        return {}
    vals, digest = {}, {}
    with open(path) as f:
        for line in f:
            parts = line.split()
            if len(parts) == 3 and parts[0] == "sources_sha256":
                digest[parts[1]] = parts[2]
            elif len(parts) == 3 and parts[0] == "traffic_bytes":
                vals[parts[1]] = float(parts[2])
    return {k: v for k, v in vals.items() if k in TRAFFIC_SOURCES and digest.get(k) == sources_hash(k)}


def host_info():
    model = platform.processor() or "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count() or 1
    return model, os.cpu_count() or 1, usable


# ---------------------------------------------------------------- references

def lib_gram_folds(X, y, K, seed):
    """FP64 per-fold sums of the rows by library products (numpy BLAS), in
    row chunks: the exact statistics the oracle's paths run on at full size."""
    import numpy as np
    import oracle
    n, p = X.shape
    fid = oracle.fold_ids(seed, n, K) if K > 1 else np.zeros(n, dtype=np.uint8)
    G = np.zeros((K, p, p)); b = np.zeros((K, p)); yy = np.zeros(K); nk = np.zeros(K, dtype=np.int64)
    chunk = 1 << 18
    for r0 in range(0, n, chunk):
        Xc = X[r0:r0 + chunk].astype(np.float64)
        yc = y[r0:r0 + chunk]
        fc = fid[r0:r0 + chunk]
        for k in range(K):
            m = fc == k
            if not m.any():
                continue
            Xk = Xc[m]
            G[k] += Xk.T @ Xk
            b[k] += Xk.T @ yc[m]
            yy[k] += float(yc[m] @ yc[m])
            nk[k] += int(m.sum())
    return G, b, yy, nk


def errors_vs_oracle(st, pens, lam, groups, betas, tol=1e-10):
    """Coefficient error (standardised scale, relative to each solution's
    largest coefficient, lambda 2..L), objective error (the oracle's f at the
    GPU's beta minus at its own, relative) and the active-set mismatches of
    the mixed-precision rule (margin < 1e-5) per form, against the oracle's
    path pipeline (Jacobi d, OEM loops) on statistics `st`."""
    import numpy as np
    import oracle
    t0 = time.perf_counter()
    ref = oracle.fit_from_stats(st, pens, lam, groups=groups, tol=tol)
    t_ref = time.perf_counter() - t0
    out = {}
    for form, b in betas.items():
        bs = b * st["s"][None, None, :]
        ce, oe, mism, undecidable = 0.0, 0.0, 0, 0
        for q, pen in enumerate(pens):
            P = oracle._as_pen(pen)
            for l in range(1, lam.shape[1]):
                br = ref["beta_std"][q, l]
                sc = np.abs(br).max()
                if sc > 0:
                    ce = max(ce, float(np.abs(bs[q, l] - br).max() / sc))
                fr = ref["obj"][q, l]
                fg = oracle.objective(st["Gs"], st["cs"], st["yyn"], P, lam[q, l], bs[q, l], groups)
                oe = max(oe, abs(fg - fr) / max(abs(fr), 1e-300))
                diff = (bs[q, l] != 0) != (br != 0)
                if diff.any():
                    g = st["Gs"] @ br - st["cs"]
                    if P.kind in oracle.GROUP_KINDS and groups is not None:
                        # per group: | ||g_g|| - c_g lambda | / (c_g lambda)
                        gid = np.asarray(groups)
                        size = np.bincount(gid).astype(float)
                        gn = np.sqrt(np.bincount(gid, weights=g * g))
                        thr = np.sqrt(size) * lam[q, l]
                        margin = (np.abs(gn - thr) / thr)[gid]
                    else:
                        margin = np.abs(np.abs(g) - lam[q, l]) / lam[q, l]
                    mism += int(diff.sum())
                    undecidable += int((margin[diff] < 1e-5).sum())
        out[form] = dict(coef_err=ce, obj_err=oe, active_set_mismatch=mism,
                         mismatch_within_margin_rule=undecidable)
    return out, t_ref, ref


# ---------------------------------------------------------------- CPU baseline

def cpu_baseline_cv(X, y, K, seed, stats, pens, lam, groups, n_full, target_s=4.0):
    """The oracle on this host's cores: its row-loop Gram (with fold sums) on
    a bounded row sample, measured and scaled linearly to n (the loop's cost
    per row is fixed), plus its path pipeline (Jacobi d, OEM loops) for every
    (problem, penalty) path on the workload's own statistics, measured.
    Single-threaded and on all usable cores (rows split in contiguous blocks,
    paths one per thread)."""
    import numpy as np
    import oracle
    model, ncpu, usable = host_info()
    p = X.shape[1]
    # rows the single thread handles in about target_s
    t0 = time.perf_counter()
    oracle.gram_folds(np.ascontiguousarray(X[:2000]), y[:2000], K, seed)
    per_row = (time.perf_counter() - t0) / 2000
    rows1 = int(min(X.shape[0], max(2000, target_s / per_row)))
    t0 = time.perf_counter()
    oracle.gram_folds(np.ascontiguousarray(X[:rows1]), y[:rows1], K, seed)
    t_gram1 = (time.perf_counter() - t0) * n_full / rows1
    rowsN = int(min(X.shape[0], rows1 * usable))
    blocks = np.linspace(0, rowsN, usable + 1).astype(int)

    def gram_block(i):
        a, b_ = blocks[i], blocks[i + 1]
        return oracle.gram_folds(np.ascontiguousarray(X[a:b_]), y[a:b_], K, seed, row_offset=int(a))

    with ThreadPoolExecutor(usable) as ex:
        t0 = time.perf_counter()
        list(ex.map(gram_block, range(usable)))
        t_gramN = (time.perf_counter() - t0) * n_full / rowsN
    # paths: every problem (its d by Jacobi, then each penalty's path) on the
    # workload's own statistics
    def problem(st):
        d = oracle.oem_d(st["Gs"])
        for q in range(len(pens)):
            oracle.fit_path_std(st["Gs"], st["cs"], st["yyn"], d, oracle._as_pen(pens[q]), lam[q], groups,
                                tol=1e-10)

    t0 = time.perf_counter()
    problem(stats[0])
    t_path1 = (time.perf_counter() - t0) * len(stats)
    with ThreadPoolExecutor(usable) as ex:
        t0 = time.perf_counter()
        list(ex.map(problem, stats))
        t_pathN = time.perf_counter() - t0
    fits = len(stats) * len(pens)
    return dict(value=fits / (t_gramN + t_pathN), unit="fits/s", cores=usable, kind="oracle",
                sample=(f"Gram row loops on {rowsN} of {n_full} rows ({usable} threads, contiguous "
                        f"blocks; {rows1} rows single-threaded), scaled linearly to n; the {len(stats)} "
                        f"problems' paths ({len(pens)} penalties x {lam.shape[1]} lambdas, Jacobi d, OEM "
                        f"loops) on the workload's FP64 statistics, one problem per thread "
                        f"(single-threaded: the full-data problem measured, times {len(stats)})"),
                cpu_model=model, nproc=ncpu, usable_cores=usable,
                seconds_per_step=t_gramN + t_pathN,
                single_core=dict(value=fits / (t_gram1 + t_path1), unit="fits/s", cores=1,
                                 seconds_per_step=t_gram1 + t_path1, gram_s=t_gram1, paths_s=t_path1),
                all_cores=dict(gram_s=t_gramN, paths_s=t_pathN))


# ---------------------------------------------------------------- timing

def time_cv_form(oem, torch, X, y, K, form, pens, groups, nlambda, steps, warm, pipelined=True,
                 depth=CV_IN_FLIGHT):
    """Whole steps of one form, one problem in flight and (pipelined) three
    in flight on three streams and three handles: the Gram pass of step i + 1
    is enqueued before oem_cv of step i and runs beside its combination and
    d, and both run beside the paths of the steps before (the paths hold one
    CU each, 33 a step; oem_cv waits for its d, so one d launch runs at a
    time, on at most half of the CUs, beside work that finishes by itself).  Then one step split
    into phases with HIP events on the launch stream: Gram pass, first
    oem_cv (d of the 11 problems + paths + CV), a second oem_cv on the same
    statistics (paths + CV: d is kept), and the Gram pass alone back to
    back."""
    import numpy as np
    p = X.shape[1]
    g = oem.Gram(p, K, form, X.dtype, CV_SEED)
    oem.oem_gram_autotune(g.h, X, y)       # untimed; leaves the sums cleared
    stream = torch.cuda.current_stream()
    ev = lambda: torch.cuda.Event(enable_timing=True)

    def step():
        oem.oem_gram_reset(g.h)
        g.add(X, y)
        return g.cv(pens, nlambda=nlambda, lambda_min_ratio=1e-3, tol=1e-10, groups=groups, sync=False)

    for _ in range(warm):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        res = step()
    torch.cuda.synchronize()
    t_seq = time.perf_counter() - t0
    t = t_seq
    identical = None
    if pipelined:
        # the tuned workgroup count is per shape, so the extra handles use it too
        extra = [oem.Gram(p, K, form, X.dtype, CV_SEED) for _ in range(depth - 1)]
        handles = [g] + extra
        streams = [stream] + [torch.cuda.Stream() for _ in extra]

        def gram_step(i):
            st, h = streams[i % depth], handles[i % depth]
            with torch.cuda.stream(st):
                oem.oem_gram_reset(h.h)
                h.add(X, y)

        def cv_step(i):
            st, h = streams[i % depth], handles[i % depth]
            with torch.cuda.stream(st):
                return h.cv(pens, nlambda=nlambda, lambda_min_ratio=1e-3, tol=1e-10, groups=groups, sync=False)

        def run(count):
            # the Gram pass of step i + 1 is enqueued before oem_cv of step i,
            # so it runs beside step i's d instead of after it
            outs = []
            gram_step(0)
            for i in range(count):
                if i + 1 < count:
                    gram_step(i + 1)
                outs.append(cv_step(i))
            return outs

        # every handle runs at least once before the timed steps (its first
        # call sizes its buffers)
        run(max(warm, depth))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        outs = run(steps)
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        ref = res["beta"].cpu().numpy()
        identical = all(np.array_equal(r["beta"].cpu().numpy(), ref) for r in outs)
        del outs
        for h in extra:
            h.close()
    e = [ev() for _ in range(4)]
    oem.oem_gram_reset(g.h)
    e[0].record(stream)
    g.add(X, y)
    e[1].record(stream)
    res = g.cv(pens, nlambda=nlambda, lambda_min_ratio=1e-3, tol=1e-10, groups=groups, sync=False)
    e[2].record(stream)
    res2 = g.cv(pens, nlambda=nlambda, lambda_min_ratio=1e-3, tol=1e-10, groups=groups, sync=False)
    e[3].record(stream)
    torch.cuda.synchronize()
    import ctypes as C
    steps_arr = (C.c_int32 * (K + 1))()
    lib = oem.load_library()
    lib.oem_debug_lanczos_steps.restype = C.c_int
    lib.oem_debug_lanczos_steps.argtypes = [C.c_void_p, C.POINTER(C.c_int32), C.c_int32]
    nq = lib.oem_debug_lanczos_steps(g.h, steps_arr, K + 1)
    lz_steps = [int(steps_arr[i]) for i in range(max(0, min(nq, K + 1)))]
    reps = 10
    a, b = ev(), ev()
    a.record(stream)
    for _ in range(reps):
        g.add(X, y)
    b.record(stream)
    torch.cuda.synchronize()
    out = dict(ms_per_step=1e3 * t / steps, fits_per_s=(K + 1) * len(pens) * steps / t,
               sequential_ms_per_step=1e3 * t_seq / steps,
               sequential_fits_per_s=(K + 1) * len(pens) * steps / t_seq,
               pipelined=pipelined, pipelined_results_identical=identical,
               gram_ms=e[0].elapsed_time(e[1]), cv_ms=e[1].elapsed_time(e[2]),
               paths_ms=e[2].elapsed_time(e[3]), gram_only_ms=a.elapsed_time(b) / reps,
               updates=int(np.abs(res2["iters"].cpu().numpy()).sum()),
               beta=res["beta"].cpu().numpy(), lam=res["lambda_"].cpu().numpy(),
               i_min=res["i_min"].cpu().numpy(), i_1se=res["i_1se"].cpu().numpy(),
               best=int(res["best"].item()), lanczos_steps=lz_steps)
    out["derive_ms"] = max(0.0, out["cv_ms"] - out["paths_ms"])
    g.close()
    return out


def gram_roofline(x_bytes, ms, traffic, kernel):
    gbs = x_bytes / (ms * 1e-3) / 1e9
    return dict(bound="hbm", kernel=kernel, achieved=gbs, peak=HBM_PEAK_GBS, unit="GB/s",
                frac=gbs / HBM_PEAK_GBS, traffic=traffic,
                algorithmic=f"{x_bytes} B per pass: X read once and y")


def gram_mfma_side(n, p, ms, precision):
    """The same Gram pass as matrix-core work: n p (p + 1) flops per product
    (the upper triangle with the diagonal), three products for split-BF16."""
    nprod = {"split_bf16": 3, "bf16": 1, "fp64": 1}[precision]
    peak = FP64_PEAK_TFLOPS if precision == "fp64" else MFMA_BF16_PEAK_TFLOPS
    tf = nprod * float(n) * p * (p + 1) / (ms * 1e-3) / 1e12
    return dict(achieved=tf, peak=peak, unit="TFLOP/s", frac=tf / peak,
                algorithmic=f"{nprod} x n p (p + 1) flops per pass")


def path_roofline(p, updates, ms, kernel):
    tf = 2.0 * p * p * updates / (ms * 1e-3) / 1e12
    return dict(bound="alu", kernel=kernel, achieved=tf, peak=FP64_PEAK_TFLOPS, unit="TFLOP/s",
                frac=tf / FP64_PEAK_TFLOPS, traffic=None,
                algorithmic=f"2 p^2 flops per OEM update x {updates} updates (FP64 vector peak)")


def lanczos_roofline(p, steps, ms):
    flops = 2.0 * p * p * sum(abs(s) for s in steps)
    tf = flops / (ms * 1e-3) / 1e12
    return dict(bound="alu", kernel="multi-workgroup Lanczos (d of every problem)", achieved=tf,
                peak=FP64_PEAK_TFLOPS, unit="TFLOP/s", frac=tf / FP64_PEAK_TFLOPS, traffic=None,
                algorithmic=f"2 p^2 flops per Lanczos step x {sum(abs(s) for s in steps)} steps")


def run_tall_form(oem, torch, X, y, precision, steps, warm, nlambda):
    """Whole steps (reset, Gram pass, the four paths) of one form; then one
    step split into Gram / fit phases and the Gram pass alone."""
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
        res = g.fit_path(TALL_PENALTIES, nlambda=nlambda, lambda_min_ratio=1e-3, tol=1e-10,
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
    rec = [ev(), ev(), ev()]
    res = step(rec)
    torch.cuda.synchronize()
    reps = 20
    a, b = ev(), ev()
    a.record(stream)
    for _ in range(reps):
        g.add(X, y)
    b.record(stream)
    torch.cuda.synchronize()
    out = dict(ms_per_step=1e3 * t_steps / steps, fits_per_s=len(TALL_PENALTIES) * steps / t_steps,
               gram_ms=rec[0].elapsed_time(rec[1]), fit_ms=rec[1].elapsed_time(rec[2]),
               gram_only_ms=a.elapsed_time(b) / reps,
               updates=int(np.abs(res["iters"].cpu().numpy()).sum()), beta=res["beta"].cpu().numpy(),
               lam=res["lambda_"].cpu().numpy())
    g.close()
    return out


def tall_record(oem, torch, args, with_errors=True):
    """The tall multi-penalty workload: n = 1e6, p = 100, AR(1) rho = 0.5,
    FP32 X, lasso / enet / MCP / SCAD, 100 lambdas."""
    import numpy as np
    import oracle
    import workloads
    n = args.n if args.tall and args.n else 1_000_000
    p = args.p if args.tall and args.p else 100
    pr = workloads.tall_multi(n=n, p=p)
    X = torch.from_numpy(pr.X).cuda()
    y = torch.from_numpy(pr.y).cuda()
    steps = args.profile_steps or args.steps
    warm = 0 if args.profile_steps else args.warmup
    forms = [args.precision] if (args.profile_steps or args.precision == "fp64") else [args.precision, "fp64"]
    runs = {f: run_tall_form(oem, torch, X, y, f, steps, warm, args.nlambda) for f in forms}
    if args.calibrate_copy:
        Z = torch.empty_like(X)
        Z.copy_(X)
        torch.cuda.synchronize()
        del Z
    m = runs[args.precision]
    x_bytes = n * p * 4 + n * 8
    traffic = stored_traffic("tall_multi").get("gram") if args.precision == "split_bf16" else None
    rec = dict(workload="tall_multi: n=1e6 p=100 AR(1) rho=0.5 FP32 X, lasso+enet+MCP+SCAD, 100 lambdas each, "
                        "tol 1e-10", n=n, p=p,
               fits_per_s=m["fits_per_s"], ms_per_step=m["ms_per_step"], gram_ms_in_step=m["gram_ms"],
               fit_ms_in_step=m["fit_ms"], oem_updates=m["updates"],
               gram_roofline=dict(gram_roofline(x_bytes, m["gram_only_ms"], traffic,
                                                "Gram pass (split-BF16 kernel + fixed-order reduction)"),
                                  mfma=gram_mfma_side(n, p, m["gram_only_ms"], args.precision)),
               path_roofline=path_roofline(p, m["updates"], m["fit_ms"],
                                           "path kernels (+ combine, Lanczos d, lambda grid)"))
    if "fp64" in runs and args.precision != "fp64":
        f = runs["fp64"]
        rec["fp64_form"] = dict(fits_per_s=f["fits_per_s"], ms_per_step=f["ms_per_step"],
                                gram_ms_in_step=f["gram_ms"], fit_ms_in_step=f["fit_ms"],
                                gram_gbps=x_bytes / (f["gram_only_ms"] * 1e-3) / 1e9)
        rec["mixed_vs_fp64_fits"] = m["fits_per_s"] / f["fits_per_s"]
    if with_errors:
        G, b, yy, nk = lib_gram_folds(pr.X, pr.y, 1, 0)
        st = oracle.prepare(G[0], b[0], yy[0], nk[0])
        betas = {form: r["beta"] for form, r in runs.items()}
        errs, t_ref, _ = errors_vs_oracle(st, TALL_PENALTIES, runs[args.precision]["lam"], None, betas)
        rec["errors_vs_fp64_oracle"] = errs
    return rec, pr, X, y


def group_record(oem, torch, X, y, groups, pr_stats, nlambda):
    """Group MCP, group SCAD and the sparse group lasso (tau 0.5) on the
    grouped workload's full data (split-BF16 Gram, general path kernel)."""
    import numpy as np
    import oracle
    p = X.shape[1]
    with oem.Gram(p, 1, "split_bf16", X.dtype) as g:
        g.add(X, y)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = g.fit_path(GROUP_PENALTIES, nlambda=nlambda, lambda_min_ratio=1e-3, tol=1e-10, groups=groups)
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        beta = res["beta"].cpu().numpy()
        lam = res["lambda_"].cpu().numpy()
        upd = int(np.abs(res["iters"].cpu().numpy()).sum())
    out = dict(penalties="group MCP gamma 3, group SCAD gamma 3.7, sparse group lasso tau 0.5",
               fits_per_s=len(GROUP_PENALTIES) / t, ms=1e3 * t, oem_updates=upd,
               path_roofline=path_roofline(p, upd, 1e3 * t, "general path kernel"))
    if pr_stats is not None:
        errs, _, _ = errors_vs_oracle(pr_stats, GROUP_PENALTIES, lam, groups, {"split_bf16": beta})
        out["errors_vs_fp64_oracle"] = errs["split_bf16"]
    return out


def out_of_core_record(oem, torch, Xh, yh, device_gram_ms):
    """oem_gram_host over the tall workload's X in host memory (pageable
    numpy array, then pinned), 131072-row chunks: the PCIe-inclusive rate."""
    import numpy as np
    n, p = Xh.shape
    x_bytes = n * p * 4 + n * 8
    out = dict(chunk_rows=131072, x_bytes=x_bytes, device_resident_gram_ms=device_gram_ms)
    with oem.Gram(p, 1, "split_bf16", torch.float32) as g:
        for label, Xs in [("pageable", Xh), ("pinned", torch.from_numpy(Xh).pin_memory())]:
            g.add_host(Xs, yh, chunk_rows=131072)        # warm (allocates the staging)
            torch.cuda.synchronize()
            oem.oem_gram_reset(g.h)
            t0 = time.perf_counter()
            g.add_host(Xs, yh, chunk_rows=131072)
            torch.cuda.synchronize()
            t = time.perf_counter() - t0
            out[label] = dict(ms=1e3 * t, gbps=x_bytes / t / 1e9)
    return out


def sparse_record(oem, torch):
    """The paper's sparse example: n = 1e5, p = 200, 1% density; the CSR
    Gram pass against the dense pass on the densified rows, then lasso and
    group lasso (groups of 5) paths, 100 lambdas."""
    import numpy as np
    from scipy import sparse
    import workloads
    sp = workloads.sparse_rows()
    n, p = len(sp.rowptr) - 1, sp.p
    rp, ci, va, yv = (torch.from_numpy(a).cuda() for a in (sp.rowptr, sp.col, sp.val, sp.y))
    Xd = torch.from_numpy(np.ascontiguousarray(
        sparse.csr_matrix((sp.val, sp.col, sp.rowptr), shape=(n, p)).toarray())).cuda()
    ev = lambda: torch.cuda.Event(enable_timing=True)
    stream = torch.cuda.current_stream()
    out = dict(n=n, p=p, nnz=int(sp.rowptr[-1]))
    groups = (np.arange(p) // 5).astype(np.int32)
    with oem.Gram(p, 1, "fp64", torch.float64) as g:
        for label, fn in [("csr", lambda: g.add_csr(rp, ci, va, yv)), ("dense", lambda: g.add(Xd, yv))]:
            fn()
            reps = 20
            a, b = ev(), ev()
            a.record(stream)
            for _ in range(reps):
                fn()
            b.record(stream)
            torch.cuda.synchronize()
            out[f"{label}_gram_ms"] = a.elapsed_time(b) / reps
        oem.oem_gram_reset(g.h)
        g.add_csr(rp, ci, va, yv)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = g.fit_path(["lasso", "grp_lasso"], nlambda=100, lambda_min_ratio=1e-3, tol=1e-10, groups=groups)
        torch.cuda.synchronize()
        out["paths_ms"] = 1e3 * (time.perf_counter() - t0)
    out["csr_bytes_per_pass"] = int(sp.rowptr[-1]) * 12 + (n + 1) * 8 + n * 8
    return out


def logistic_record(oem, torch):
    """Logistic regression (proximal Newton, OEM inner loop) on the tall
    shape n = 1e6, p = 100 (AR(1) rho 0.5, 10 nonzero coefficients x 0.5):
    a 100-lambda lasso path, exact Hessian and the bound 1/4."""
    import numpy as np
    import workloads
    pr = workloads.logistic(n=1_000_000, p=100)
    X = torch.from_numpy(pr.X).cuda()
    y = torch.from_numpy(pr.y).cuda()
    out = dict(n=1_000_000, p=100, nlambda=100)
    for label, bound in [("exact_hessian", False), ("hessian_bound", True)]:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = oem.logistic_path(X, y, ["lasso"], nlambda=100, lambda_min_ratio=1e-2, tol=1e-10,
                              newton_tol=1e-8, newton_maxit=100 if not bound else 2000,
                              hessian_bound=bound)
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        nt = r["newton"].cpu().numpy()
        out[label] = dict(fits_per_s=1.0 / t, ms=1e3 * t, newton_steps=int(np.abs(nt).sum()),
                          max_kkt=float(r["kkt"].cpu().numpy().max()), status=int(r["status"]))
    return out


def guarded(fn, *a, **k):
    try:
        return fn(*a, **k)
    except Exception as e:      # a sub-record never takes the main line down
        return {"error": f"{type(e).__name__}: {e}"}


def cv_main(args):
    """The default line: the grouped 10-fold CV workload."""
    import numpy as np
    import torch
    import paper_1801_09661_amd as oem
    import oracle
    import workloads

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    oem.load_library()
    n = args.n or 2_000_000
    p = args.p or 500
    K = 10
    pr = workloads.cv_grouped(n=n, p=p)
    X = torch.from_numpy(pr.X).cuda()
    y = torch.from_numpy(pr.y).cuda()
    groups = pr.groups
    torch.cuda.synchronize()
    steps = args.profile_steps or args.steps
    warm = 0 if args.profile_steps else args.warmup
    forms = [args.precision] if (args.profile_steps or args.precision == "fp64") else [args.precision, "fp64"]
    pipelined = not (args.sequential or args.profile_steps)
    runs = {f: time_cv_form(oem, torch, X, y, K, f, CV_PENALTIES, groups, args.nlambda, steps, warm, pipelined,
                            args.in_flight)
            for f in forms}
    if args.calibrate_copy:
        Z = torch.empty_like(X)
        Z.copy_(X)
        torch.cuda.synchronize()
        del Z
    m = runs[args.precision]
    x_bytes = n * p * X.element_size() + n * 8
    traffic = stored_traffic("cv_grouped").get("gram") if args.precision == "split_bf16" else None
    roofs = dict(gram=dict(gram_roofline(x_bytes, m["gram_only_ms"], traffic,
                                         "Gram pass with fold sums (split-BF16 kernels + fixed-order reduction)"),
                           mfma=gram_mfma_side(n, p, m["gram_only_ms"], args.precision)),
                 lanczos=lanczos_roofline(p, m["lanczos_steps"], m["derive_ms"]),
                 paths=path_roofline(p, m["updates"], m["paths_ms"], "path kernels + CV error"))
    phase_ms = dict(gram=m["gram_ms"], lanczos=m["derive_ms"], paths=m["paths_ms"])
    dominant = max(phase_ms, key=phase_ms.get)
    out = {
        "metric": METRIC,
        "value": m["fits_per_s"],
        "unit": "fits/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warm,
        "ms_per_step": m["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPE[args.precision],
        "data": "synthetic",
        "config": {"workload": "cv_grouped: n=2e6 p=500 AR(1) rho=0.3 FP32 X, 10 hashed folds, 50 groups "
                               "of 10 (5 active), group lasso+lasso+MCP, 100 lambdas, tol 1e-10",
                   "n": n, "p": p, "folds": K, "penalties": len(CV_PENALTIES), "nlambda": args.nlambda,
                   "precision": args.precision},
        "pipeline": (f"{args.in_flight} CV problems in flight on {args.in_flight} streams: the Gram pass of "
                     "step i + 1 enqueued before oem_cv of step i (beside its d), both beside the paths of the "
                     "steps before; every step is a whole Gram pass + oem_cv" if pipelined
                     else "one CV problem in flight"),
        "sequential": dict(ms_per_step=m["sequential_ms_per_step"], fits_per_s=m["sequential_fits_per_s"]),
        "pipelined_results_identical": m["pipelined_results_identical"],
        "phase_ms": phase_ms,
        "gram_gbps": x_bytes / (m["gram_only_ms"] * 1e-3) / 1e9,
        "oem_updates": m["updates"],
        "lanczos_steps": m["lanczos_steps"],
        "roofline": dict(roofs[dominant], phase=dominant),
        "gram_roofline": roofs["gram"],
        "phase_rooflines": roofs,
    }
    if "fp64" in runs and args.precision != "fp64":
        f = runs["fp64"]
        out["fp64_form"] = dict(fits_per_s=f["fits_per_s"], ms_per_step=f["ms_per_step"],
                                sequential=dict(ms_per_step=f["sequential_ms_per_step"],
                                                fits_per_s=f["sequential_fits_per_s"]),
                                phase_ms=dict(gram=f["gram_ms"], lanczos=f["derive_ms"], paths=f["paths_ms"]),
                                gram_tflops=2.0 * n * p * (p + 1) / 2 / (f["gram_only_ms"] * 1e-3) / 1e12)
        out["fp64_form"]["gram_roofline"] = dict(
            bound="mfma", kernel="FP64 Gram pass (v_mfma_f64_16x16x4f64)",
            achieved=out["fp64_form"]["gram_tflops"], peak=FP64_PEAK_TFLOPS, unit="TFLOP/s",
            frac=out["fp64_form"]["gram_tflops"] / FP64_PEAK_TFLOPS, traffic=None,
            algorithmic="n p (p + 1) flops per pass (upper triangle with the diagonal, 2 per product)")
        out["mixed_vs_fp64_fits"] = m["fits_per_s"] / f["fits_per_s"]
        out["mixed_vs_fp64_fits_sequential"] = m["sequential_fits_per_s"] / f["sequential_fits_per_s"]
    if args.profile_steps or args.no_extras:
        print(json.dumps(out))
        return
    # errors of the full-data paths against the oracle on the exact statistics
    G, b, yy, nk = lib_gram_folds(pr.X, pr.y, K, CV_SEED)
    full = oracle.prepare(G.sum(0), b.sum(0), yy.sum(), nk.sum())
    betas = {form: r["beta"] for form, r in runs.items()}
    errs, t_ref, _ = errors_vs_oracle(full, CV_PENALTIES, m["lam"], groups, betas)
    out["errors_vs_fp64_oracle"] = dict(errs, scope="full-data paths, 3 penalties x 100 lambdas; oracle "
                                                    "path pipeline on the FP64 statistics of the same rows")
    if not args.no_cpu_baseline:
        stats = [full] + [oracle.prepare(G.sum(0) - G[k], b.sum(0) - b[k], yy.sum() - yy[k], nk.sum() - nk[k])
                          for k in range(K)]
        out["cpu_baseline"] = cpu_baseline_cv(pr.X, pr.y, K, CV_SEED, stats, CV_PENALTIES, m["lam"], groups, n)
    del G, b
    out["group_penalties"] = guarded(group_record, oem, torch, X, y, groups, full, args.nlambda)
    del X, y, pr
    torch.cuda.empty_cache()
    tall = guarded(tall_record, oem, torch, args)
    if isinstance(tall, tuple):
        rec, tpr, tX, ty = tall
        out["tall_multi"] = rec
        out["out_of_core"] = guarded(out_of_core_record, oem, torch, tpr.X, tpr.y, rec["gram_ms_in_step"])
        del tX, ty, tpr
        torch.cuda.empty_cache()
    else:
        out["tall_multi"] = tall
    out["sparse"] = guarded(sparse_record, oem, torch)
    out["logistic"] = guarded(logistic_record, oem, torch)
    print(json.dumps(out))


def tall_main(args):
    """The tall multi-penalty workload as the main line."""
    import torch
    import paper_1801_09661_amd as oem
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    oem.load_library()
    rec, pr, X, y = tall_record(oem, torch, args, with_errors=not (args.profile_steps or args.no_extras))
    steps = args.profile_steps or args.steps
    out = {"metric": METRIC, "value": rec["fits_per_s"], "unit": "fits/s", "n_gpus": 1, "steps": steps,
           "warmup": 0 if args.profile_steps else args.warmup, "ms_per_step": rec["ms_per_step"],
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": DTYPE[args.precision],
           "data": "synthetic",
           "config": {"workload": rec.pop("workload"), "n": rec["n"], "p": rec["p"], "penalties": 4,
                      "nlambda": args.nlambda, "precision": args.precision}}
    dom = rec["gram_roofline"] if rec["gram_ms_in_step"] >= rec["fit_ms_in_step"] else rec["path_roofline"]
    out["roofline"] = dom
    out.update(rec)
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
    # the Gram passes alone (one handle per problem, back to back on one
    # stream, events around them): the HBM-bound part of a step
    stream = torch.cuda.current_stream()
    gram_ms, x_bytes = 0.0, 0
    for X, y in dev:
        n, p = X.shape
        with oem.Gram(p, 1, args.precision, X.dtype) as g:
            g.add(X, y)
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            g.add(X, y)
            b.record(stream)
            torch.cuda.synchronize()
            gram_ms += a.elapsed_time(b)
        x_bytes += n * p * X.element_size() + 8 * n
    rest_ms = max(main_run["ms_per_step"] - gram_ms, 1e-9)
    psq = sum(X.shape[1] ** 2 for X, _ in dev) / len(dev)
    # Most of the passes' time is matrix-core work: a problem's pass is bound
    # by the matrix cores when its products outweigh its bytes at the peak
    # rates (p above about 420 for split-BF16), and those problems carry most
    # of the flops.  The line reports the passes against the matrix-core peak,
    # with the HBM figure and the per-problem roofline time beside it.
    g_hbm = gram_roofline(x_bytes, gram_ms, None, "Gram passes of the 64 problems (one after another)")
    nprod = {"split_bf16": 3, "bf16": 1, "fp64": 1}[args.precision]
    mpeak = FP64_PEAK_TFLOPS if args.precision == "fp64" else MFMA_BF16_PEAK_TFLOPS
    pflops = [nprod * float(X.shape[0]) * X.shape[1] * (X.shape[1] + 1) for X, _ in dev]
    pbytes = [float(X.shape[0]) * X.shape[1] * X.element_size() + 8.0 * X.shape[0] for X, _ in dev]
    t_roof = [max(fb / (HBM_PEAK_GBS * 1e9), ff / (mpeak * 1e12)) for ff, fb in zip(pflops, pbytes)]
    g_tf = sum(pflops) / (gram_ms * 1e-3) / 1e12
    g_roof = dict(bound="mfma", kernel="Gram passes of the 64 problems (one after another)", achieved=g_tf,
                  peak=mpeak, unit="TFLOP/s", frac=g_tf / mpeak, traffic=None,
                  algorithmic=f"{nprod} x n p (p + 1) flops per problem (the upper triangle with the diagonal, "
                              f"2 per product; {nprod} products), {sum(pflops):.4e} in all",
                  mfma_bound_problems=sum(1 for ff, fb in zip(pflops, pbytes)
                                          if ff / (mpeak * 1e12) > fb / (HBM_PEAK_GBS * 1e9)),
                  roofline_ms=1e3 * sum(t_roof), frac_of_roofline_time=1e3 * sum(t_roof) / gram_ms,
                  hbm=dict(achieved=g_hbm["achieved"], peak=HBM_PEAK_GBS, unit="GB/s", frac=g_hbm["frac"],
                           algorithmic=g_hbm["algorithmic"]))
    p_roof = dict(bound="alu", kernel="d and path kernels of the 64 problems (the rest of the step)",
                  achieved=2.0 * psq * main_run["updates"] / (rest_ms * 1e-3) / 1e12, peak=FP64_PEAK_TFLOPS,
                  unit="TFLOP/s", traffic=None,
                  algorithmic="2 p^2 flops per OEM update (mean p^2 of the problems) x updates")
    p_roof["frac"] = p_roof["achieved"] / FP64_PEAK_TFLOPS
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
        "roofline": g_roof if gram_ms >= rest_ms else p_roof,
        "gram_roofline": g_roof,
        "gram_ms_of_step": gram_ms,
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
        errs, worst = [], None
        for i, (bm, bf) in enumerate(zip(main_run["beta"], f64["beta"])):
            scale = np.maximum(np.abs(bf).max(axis=2), 1e-300)
            e = (np.abs(bm - bf).max(axis=2) / scale)[:, 1:]
            errs.append(float(e.max()))
            if worst is None or errs[-1] > worst["coef_err"]:
                q, l = np.unravel_index(int(np.argmax(e)), e.shape)
                j = int(np.argmax(np.abs(bm[q, l + 1] - bf[q, l + 1])))
                worst = dict(coef_err=errs[-1], problem=i, p=int(bf.shape[2]), lambda_index=int(l + 1),
                             coord=j, beta_fp64=float(bf[q, l + 1, j]), beta_mixed=float(bm[q, l + 1, j]),
                             max_abs_beta=float(scale[q, l + 1]),
                             active_set_mismatch=int(np.count_nonzero((bm[:, 1:] != 0) != (bf[:, 1:] != 0))))
        out["mixed_coef_err_vs_fp64_form_max"] = max(errs)
        out["mixed_coef_err_vs_fp64_form_median"] = float(np.median(errs))
        out["mixed_coef_err_worst_problem"] = worst
    if not args.no_cpu_baseline and not args.profile_steps:
        out["cpu_baseline"] = cpu_baseline_batch(shapes)
    print(json.dumps(out))


def cpu_baseline_batch(shapes, pmax=256):
    """The oracle (row-loop Gram, Jacobi d, lasso path of 100 lambdas) on
    the batch's problems with p <= pmax (the larger ones take the oracle
    minutes each), one problem per thread on all cores and single-threaded;
    fits/s on that sample."""
    import numpy as np
    import oracle
    import workloads
    model, ncpu, usable = host_info()
    sample = [(i, n, p) for i, (n, p) in enumerate(shapes) if p <= pmax]
    probs = [workloads.batched_uneven_problem(i, n, p) for i, n, p in sample]

    def fit(pr):
        oracle.fit(pr.X, pr.y, ["lasso"], nlambda=100, lambda_min_ratio=1e-3, tol=1e-10)

    t0 = time.perf_counter()
    fit(probs[0])
    t1 = time.perf_counter() - t0
    with ThreadPoolExecutor(usable) as ex:
        t0 = time.perf_counter()
        list(ex.map(fit, probs))
        tN = time.perf_counter() - t0
    return dict(value=len(probs) / tN, unit="fits/s", cores=usable, kind="oracle",
                sample=f"the {len(probs)} of {len(shapes)} problems with p <= {pmax} (whole fits: row-loop "
                       f"Gram, Jacobi d, lasso path of 100 lambdas), one problem per thread",
                cpu_model=model, nproc=ncpu,
                single_core=dict(value=1.0 / t1, unit="fits/s", cores=1,
                                 sample=f"problem {sample[0][0]} (n={sample[0][1]}, p={sample[0][2]})"))


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
    t_oracle = time.perf_counter()
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
        "slowest_device": [dict(id=int(d["id"]), p=reqs[d["id"]].p, n=reqs[d["id"]].n,
                                penalty=reqs[d["id"]].penalty, nfolds=reqs[d["id"]].nfolds,
                                device_ms=float((d["t_done"] - d["t_admit"]) * 1e3))
                           for d in sorted(done, key=lambda d: d["t_admit"] - d["t_done"])[:6]],
        "device_s_total": float(dev.sum()),
        "cpu_baseline": dict(value=len(sample) / max(time.perf_counter() - t_oracle, 1e-9), unit="requests/s",
                             cores=1, kind="oracle",
                             sample=f"{len(sample)} plain fit requests with p <= 120, n <= 60000 (row-loop "
                                    "Gram, Jacobi d, one 100-lambda path each), one thread",
                             cpu_model=host_info()[0], nproc=host_info()[1]),
        "dtype": "split-bf16 Gram (f32 acc, f64 reduce) + f64 paths", "data": "synthetic",
        "config": {"workload": f"serving: {args.requests} requests, Poisson {args.rate}/s, p in [10,1000], "
                               "n in [1e4,1e6], AR(1) rho~U(0,0.8) (8 levels), lasso/MCP/SCAD/group lasso, "
                               "20% 5-fold CV, 100 lambdas", "slots": args.slots,
                                   "hw_queues": os.environ.get("GPU_MAX_HW_QUEUES")},
    }
    print(json.dumps(out))



def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    if args.in_flight < 1:
        print(json.dumps({"error": "--in-flight must be >= 1"}))
        sys.exit(2)
    if args.serve:
        # one hardware queue per worker stream (HIP's default is 4), set
        # before the runtime starts
        os.environ["GPU_MAX_HW_QUEUES"] = str(min(32, max(4, args.slots)))
        return serve_main(args)
    if args.batch:
        return batch_main(args)
    if args.tall:
        return tall_main(args)
    return cv_main(args)


if __name__ == "__main__":
    main()
