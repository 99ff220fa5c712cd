"""Benchmark: LSE/GLS solves/s at FP64 backward error <= 1e-14, mixed-precision
refinement vs the all-FP64 GPU path, on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--workload NAME]

Default line (--workload headline): the batched workload, 2000 LSE/GLS
instances of uneven size (seed 4), solved per step by the persistent batched
path with FP32 factors and classical refinement (instances that do not
certify continue in FP64), against the all-FP64 persistent path on the same
instances; a solve counts only if it certifies berr <= 1e-14.  The line
carries two sub-records, each mixed precision against the FP64 direct path:
the single large LSE (A 4096 x 2048, kappa 1e4, B 256 x 2048; FP32 and BF16
factorizations with classical IR) and the single large GLS (W 4096 x 1024,
V 4096 x 4096 with kappa 1e6; FP16 factorization with GMRES-IR and the
escalation ladder).  Inputs are synthetic and resident in HBM before timing
starts.  The other workloads (--workload) print a line of their own.

Prints one JSON line (the solver runs on one GPU).
"""
from __future__ import annotations

import argparse
import gc
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "LSE/GLS solves/s at FP64 backward error <=1e-14: mixed-IR vs plain FP64, 1 GPU"
WORKLOAD = "single LSE, A 4096x2048 kappa(A)=1e4 (U diag(s) V^T), B 256x2048 N(0,1), b,d N(0,1), seed 2"
PEAK = {"fp32": 157.3, "fp64": 78.6, "bf16": 2500.0, "fp16": 2500.0}   # dense MFMA TFLOP/s
HBM_PEAK = 8000.0                                                     # GB/s
COPY_BYTES = 256 << 20            # calibration copy for the hardware byte counters
# Kernels whose roofline can be reported, with their bound.  The panel kernel
# counts the Householder flops of its panel (2 mr jb^2 - 2 jb^3 / 3) against
# the FP64 peak (its arithmetic is FP64 whatever the storage precision); the
# GEMV kernels count one read of their matrix against the HBM peak.
KERNELS = {
    "panel_final_y": ("k_panel_final_y", "mfma", 78.6, "TFLOP/s"),
    "panel_cholpass": ("k_panel_cholpass", "mfma", 78.6, "TFLOP/s"),
    "wy_u": ("k_wy_u", "mfma", None, "TFLOP/s"),
    "wy_t": ("k_wy_t", "mfma", None, "TFLOP/s"),
    "dual_gemv": ("k_dual_gemv", "hbm", HBM_PEAK, "GB/s"),
    "agg_gemv": ("k_gemv_tv / k_gemv_n (aggregated reflector blocks)", "hbm", HBM_PEAK, "GB/s"),
}
KERNEL_SOURCES = ["paper_2406_16499_amd/csrc/qr.hip", "paper_2406_16499_amd/csrc/wg64.hpp",
                  "paper_2406_16499_amd/csrc/vec.hip", "paper_2406_16499_amd/csrc/blas.hip",
                  "paper_2406_16499_amd/csrc/gemv.hpp", "paper_2406_16499_amd/csrc/common.hpp",
                  "paper_2406_16499_amd/csrc/engine.hpp"]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--prec", default="fp32")
    ap.add_argument("--m", type=int, default=4096)
    ap.add_argument("--n", type=int, default=2048)
    ap.add_argument("--p", type=int, default=256)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--kernel", default="panel_final_y", choices=sorted(KERNELS))
    ap.add_argument("--workload", default="headline",
                    choices=["headline", "lse-large", "gls-large", "lse-wide", "gls-tall", "paper-grid",
                             "lse-factored", "batched"],
                    help="headline (default): the batched workload with the large LSE and GLS as "
                         "sub-records; lse-large: the single 4096x2048x256 LSE; gls-large: the "
                         "4096x1024x4096 GLS with GMRES-IR; lse-wide: LSE 2048x4096x2560 (n > m) "
                         "with GMRES-IR; gls-tall: GLS 4096x2560x2048 (n > p) with GMRES-IR; "
                         "paper-grid: the paper's experiment shapes against the GPU FP64 path; "
                         "lse-factored: the default LSE factored once, solves with new right-hand sides; "
                         "batched: the 2000-instance mixed LSE/GLS workload")
    ap.add_argument("--grid", default="E1,E2,E3", help="paper-grid: experiments to run")
    ap.add_argument("--grid-n", default="", help="paper-grid: only these n (comma-separated)")
    ap.add_argument("--count", type=int, default=2000, help="instances of the batched workload")
    ap.add_argument("--workers", type=int, default=8, help="batch workers (streams)")
    ap.add_argument("--no-workers", action="store_true",
                    help="batched workload: skip the per-instance worker runs (context lines)")
    return ap.parse_args()


BATCH_SOURCES = ["paper_2406_16499_amd/csrc/batch.hip", "paper_2406_16499_amd/csrc/common.hpp",
                 "paper_2406_16499_amd/csrc/engine.hpp"]


def source_hash(files=None):
    import hashlib
    hsh = hashlib.sha256()
    for f in (files or KERNEL_SOURCES):
        with open(os.path.join(ROOT, f), "rb") as fh:
            hsh.update(fh.read())
    return hsh.hexdigest()[:16]


def traffic_per_launch(kernel, files=None):
    """HBM bytes per launch from the committed hardware-counter summary, if it
    was taken on the current kernel sources (else None)."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_traffic.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    if kv.get("source_hash") != source_hash(files):
        return None
    try:
        return float(kv["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def time_solves(h, lsq, torch, tensors, opts, steps, warmup, kernel=None):
    A, B, b, d = tensors
    m, n = A.shape
    p = B.shape[0]
    x, r, v = lsq.empty(n), lsq.empty(m), lsq.empty(p)
    last = None
    for _ in range(warmup):
        rc, res = h.lse_solve(A, B, b, d, x, r, v, opts)
        last = res
    torch.cuda.synchronize()
    if kernel:
        h.timer_enable(kernel)
    t0 = time.perf_counter()
    ok = 0
    results = []
    for _ in range(steps):
        rc, res = h.lse_solve(A, B, b, d, x, r, v, opts)
        results.append(res.as_dict())
        if rc == 0 and res.berr_max <= 1e-14:
            ok += 1
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    timing = None
    if kernel:
        timing = h.timer_read()
        h.timer_enable(None)
    return dt, ok, results, timing


def cpu_baseline(prob, seconds):
    """The FP64 oracle (null-space method via GRQ) on the same workload."""
    from oracle import direct
    try:
        import threadpoolctl
        info = threadpoolctl.threadpool_info()
        cores = max([i.get("num_threads", 1) for i in info] or [os.cpu_count() or 1])
    except Exception:
        cores = os.cpu_count() or 1
    t0 = time.perf_counter()
    count = 0
    while True:
        direct.lse_solve(prob.A, prob.B, prob.b, prob.d)
        count += 1
        if time.perf_counter() - t0 >= seconds or count >= 50:
            break
    dt = time.perf_counter() - t0
    return {"value": count / dt, "unit": "solves/s", "cores": int(cores), "kind": "oracle",
            "sample": f"{count} full solves of the benchmark LSE (FP64 null-space GRQ oracle, numpy/scipy LAPACK) in {dt:.1f} s"}


def cpu_baseline_batch(probs, seconds):
    """The oracle (FP64 null-space / Paige solves) on the first instances of
    the batch, for about `seconds` of host time."""
    from oracle import direct
    try:
        import threadpoolctl
        info = threadpoolctl.threadpool_info()
        cores = max([i.get("num_threads", 1) for i in info] or [os.cpu_count() or 1])
    except Exception:
        cores = os.cpu_count() or 1
    t0 = time.perf_counter()
    count = 0
    for P in probs:
        if P.kind == "lse":
            direct.lse_solve(P.A, P.B, P.b, P.d)
        else:
            direct.gls_solve(P.W, P.V, P.d)
        count += 1
        if time.perf_counter() - t0 >= seconds:
            break
    dt = time.perf_counter() - t0
    return {"value": count / dt, "unit": "solves/s", "cores": int(cores), "kind": "oracle",
            "sample": f"the first {count} instances of the batch (FP64 oracle, numpy/scipy LAPACK) in {dt:.1f} s"}


BATCH_WORKLOAD = ("2000 instances, 50/50 LSE/GLS; LSE m~U[64,1024], n~U[32,m/2], p~U[4,n/4], "
                  "GLS mirrored; A,B (W,V) = U diag(s) V^T, kappa log-U[1e1,1e8]; RHS N(0,1); seed 4")


def schedule_summary(tl):
    """Work-group time of the last persistent call, from the per-instance
    device clocks (ms): the FP32 attempts (split into factorization and
    refinement, and the part spent on instances that then escalated), the
    FP64 attempts, and when the last attempt of each kind ended."""
    import numpy as np
    f32, f64 = tl[:, 0, :], tl[:, 1, :]
    has32, has64 = ~np.isnan(f32[:, 0]), ~np.isnan(f64[:, 0])
    esc = has32 & has64

    def busy(a, m):
        return float(np.sum(a[m, 2] - a[m, 0])) if m.any() else 0.0
    return {
        "fp32_attempts": int(has32.sum()), "fp64_attempts": int(has64.sum()),
        "fp32_factor_ms": float(np.sum(f32[has32, 1] - f32[has32, 0])) if has32.any() else 0.0,
        "fp32_refine_ms": float(np.sum(f32[has32, 2] - f32[has32, 1])) if has32.any() else 0.0,
        "fp32_on_escalated_ms": busy(f32, esc),
        "fp64_factor_ms": float(np.sum(f64[has64, 1] - f64[has64, 0])) if has64.any() else 0.0,
        "fp64_refine_ms": float(np.sum(f64[has64, 2] - f64[has64, 1])) if has64.any() else 0.0,
        "fp32_last_end_ms": float(np.nanmax(f32[:, 2])) if has32.any() else None,
        "fp64_first_start_ms": float(np.nanmin(f64[:, 0])) if has64.any() else None,
        "fp64_last_end_ms": float(np.nanmax(f64[:, 2])) if has64.any() else None,
        "unit": "work-group ms (sums) / ms from the first start (ends)",
    }


# The launch shape for batches whose instances mostly certify at FP32: the
# FP64 rung on 1/16 of the compute units, no instance FP64 first (the shipped
# table is tuned for the headline recipe, where about 40% need FP64).
def batched_regime(args, kappa_max):
    """The batched recipe with both condition numbers log-uniform up to
    kappa_max, mixed against all-FP64 on the same instances; a solve counts
    only if it certifies.  The handle carries the shipped launch-shape table,
    whose entry each call picks by the escalation fraction of the call before
    (a new handle starts with the entry for any regime: the first warm-up
    call's)."""
    import torch
    from paper_2406_16499_amd import lsq
    from paper_2406_16499_amd import workloads as wl
    probs = list(wl.batch_instances(seed=4, count=args.count, kappa_max=kappa_max))
    keep, descs = [], []
    for P in probs:
        if P.kind == "lse":
            t = tuple(lsq.colmajor(a) for a in (P.A, P.B, P.b, P.d))
            x = lsq.empty(P.shape[1])
            descs.append(lsq.make_problem("lse", t, x))
            keep.append((t, x))
        else:
            t = tuple(lsq.colmajor(a) for a in (P.W, P.V, P.d))
            x, y = lsq.empty(P.shape[1]), lsq.empty(P.shape[2])
            descs.append(lsq.make_problem("gls", t, x, y))
            keep.append((t, x, y))
    del probs
    arr = lsq.problem_array(descs)
    torch.cuda.synchronize()
    gc.collect()
    h = lsq.Handle(load_selector=False)
    h.set_batch_mode("persistent")

    def run(opts):
        for _ in range(args.warmup):
            h.lsq_solve_batched(arr, opts)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        results = [h.lsq_solve_batched(arr, opts, raw=True)[1] for _ in range(args.steps)]
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        ok = sum(1 for res in results for r in res if r.info == 0 and r.berr_max <= 1e-14)
        rungs = {}
        for r in results[-1]:
            key = f"{lsq.PREC_NAME.get(r.prec_used, r.prec_used)}/{lsq.SOLVER_NAME.get(r.solver_used, r.solver_used)}"
            rungs[key] = rungs.get(key, 0) + 1
        return dt, ok, rungs

    dt, ok, rungs = run(lsq.default_opts(prec="fp32", solver="ir", escalate=1))
    escalation = h.dbg_batch_regime()
    dt64, ok64, _ = run(lsq.default_opts(prec="fp64", solver="direct"))
    h.close()
    del keep, descs, arr
    gc.collect()
    value, value64 = ok / dt, ok64 / dt64
    return {"value": value, "unit": "solves/s", "ms_per_step": 1000.0 * dt / args.steps,
            "config": {"workload": BATCH_WORKLOAD.replace("1e8", f"{kappa_max:g}"), "count": args.count,
                       "kappa_max": kappa_max,
                       "schedule": "shipped table, entry picked by the previous call's escalation fraction"},
            "escalation_fraction": escalation,
            "fp64_direct": {"value": value64, "unit": "solves/s", "ms_per_step": 1000.0 * dt64 / args.steps},
            "speedup_vs_fp64": value / value64 if value64 > 0 else None,
            "certified_fraction": ok / (args.count * args.steps), "rungs_used": rungs}


def batched(args):
    """The batched workload: every instance solved per step, a solve counting
    only if it certifies berr <= 1e-14."""
    import torch
    from paper_2406_16499_amd import lsq
    from paper_2406_16499_amd import workloads as wl
    t0 = time.perf_counter()
    probs = list(wl.batch_instances(seed=4, count=args.count))
    keep, descs = [], []
    for P in probs:
        if P.kind == "lse":
            t = tuple(lsq.colmajor(a) for a in (P.A, P.B, P.b, P.d))
            x = lsq.empty(P.shape[1])
            descs.append(lsq.make_problem("lse", t, x))
            keep.append((t, x))
        else:
            t = tuple(lsq.colmajor(a) for a in (P.W, P.V, P.d))
            x, y = lsq.empty(P.shape[1]), lsq.empty(P.shape[2])
            descs.append(lsq.make_problem("gls", t, x, y))
            keep.append((t, x, y))
    torch.cuda.synchronize()
    gen_s = time.perf_counter() - t0
    # the ~8000 tensors of the instances would make every full garbage
    # collection of the interpreter a ~45 ms pause inside a timed call:
    # collect once and move them out of the collector's generations
    gc.collect()
    gc.freeze()
    # the descriptors marshalled once, as a C caller would hold them
    arr = lsq.problem_array(descs)
    h = lsq.Handle()
    h.lib.lsq_set_batch_workers(h.h, args.workers)

    def run(opts, steps, warmup, mode="persistent", kernel=None):
        h.set_batch_mode(mode)
        for _ in range(warmup):
            h.lsq_solve_batched(arr, opts)
        torch.cuda.synchronize()
        if kernel:
            h.timer_enable(kernel)
        t1 = time.perf_counter()
        results = []
        for _ in range(steps):
            rc, res = h.lsq_solve_batched(arr, opts, raw=True)
            results.append(res)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t1
        # (the per-result bookkeeping stays out of the timed region)
        ok, rungs = 0, {}
        for res in results:
            for r in res:
                if r.info == 0 and r.berr_max <= 1e-14:
                    ok += 1
                key = f"{lsq.PREC_NAME.get(r.prec_used, r.prec_used)}/{lsq.SOLVER_NAME.get(r.solver_used, r.solver_used)}"
                rungs[key] = rungs.get(key, 0) + 1
        timing = None
        if kernel:
            timing = h.timer_read()
            h.timer_enable(None)
        h.set_batch_mode("persistent")
        return dt, ok, rungs, timing

    from paper_2406_16499_amd import selector as sel
    have_sel = os.path.exists(sel.WEIGHTS_PATH)
    # persistent launch: FP32 factors and corrections, the instances that do
    # not certify factored again in FP64 inside a second persistent launch
    mixed = lsq.default_opts(prec="fp32", solver="ir", escalate=1)
    # the FP64 rung beside the FP32 launch carries most of the mixed step
    # under the tuned schedule: its launches are the ones timed
    dt, ok, rungs, tim = run(mixed, args.steps, args.warmup, kernel="batch_esc")
    sched = schedule_summary(h.dbg_batch_timeline(len(descs)))
    dt64, ok64, _, tim64 = run(lsq.default_opts(prec="fp64", solver="direct"), args.steps,
                               args.warmup, kernel="batch_fp64")
    sched64 = schedule_summary(h.dbg_batch_timeline(len(descs)))
    # the same mixed batch captured once as a HIP graph and replayed
    plan = h.batch_plan(descs, mixed)
    for _ in range(args.warmup):
        plan.run()
    torch.cuda.synchronize()
    tg = time.perf_counter()
    resg_all = []
    for _ in range(args.steps):
        rcg, resg = plan.run(raw=True)
        resg_all.append(resg)
    torch.cuda.synchronize()
    dtg = time.perf_counter() - tg
    okg = sum(1 for resg in resg_all for r in resg if r.info == 0 and r.berr_max <= 1e-14)
    plan.close()
    # per-instance solves on the batch workers (context): the learned selector
    # picks each instance's starting rung
    auto = lsq.default_opts(prec="auto", solver="auto", escalate=1)
    if not args.no_workers:
        dts, oks, rungss, _ = run(auto, 1, 0, mode="workers")
        dtl, okl, rungsl, _ = run(mixed, 1, 0, mode="workers")
        dtw, okw, _, _ = run(lsq.default_opts(prec="fp64", solver="direct"), 1, 0, mode="workers")
    # calibration copy of known size, outside the timed regions (scales the
    # FETCH_SIZE / WRITE_SIZE counters of a profiled run)
    src = torch.empty(COPY_BYTES // 8, dtype=torch.float64, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    h.dbg_copy(dst, src, COPY_BYTES)
    del src, dst
    value = ok / dt
    value64 = ok64 / dt64
    ms, launches, flops, _ = tim
    roof = None
    if launches > 0 and ms > 0:
        achieved = (flops / launches) / (ms / launches * 1e-3) / 1e12
        roof = {"bound": "mfma", "achieved": achieved, "peak": PEAK["fp64"], "unit": "TFLOP/s",
                "frac": achieved / PEAK["fp64"],
                "traffic": traffic_per_launch("batch_esc", BATCH_SOURCES),
                "kernel": "k_batch_esc (the FP64 rung beside the FP32 launch: one launch from the start, "
                          "one more when the FP32 launch ends)",
                "launches_per_step": launches / args.steps, "avg_launch_us": 1000.0 * ms / launches,
                "alg_flops_per_launch": flops / launches,
                "flops_counted": "Householder flops of the factorizations of the instances the rung solved, "
                                 "split evenly over its launches",
                "source_hash": source_hash(BATCH_SOURCES)}
    line = {
        "metric": METRIC, "value": value, "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1000.0 * dt / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "f64 (residuals, updates) / fp32 (factorization, corrections; fp64 on escalation)",
        "data": "synthetic",
        "config": {"workload": BATCH_WORKLOAD, "count": args.count,
                   "execution": "persistent, one work-group per instance",
                   "ladder": "fp32 classical IR, then fp64", "tol": 1e-14},
        "fp64_direct": {"value": value64, "unit": "solves/s",
                        "ms_per_step": 1000.0 * dt64 / args.steps,
                        "avg_launch_us": 1000.0 * tim64[0] / max(tim64[1], 1)},
        "speedup_vs_fp64": value / value64 if value64 > 0 else None,
        "graph_replay": {"value": okg / dtg, "unit": "solves/s", "ms_per_step": 1000.0 * dtg / args.steps,
                         "api": "lsq_batch_plan_run (the mixed batch captured once as a HIP graph)",
                         "certified_fraction": okg / (args.count * args.steps)},
        "schedule": {"mixed": sched, "fp64": sched64},
        "certified_fraction": ok / (args.count * args.steps),
        "rungs_used": rungs,
        "workers_selector": None if args.no_workers else
        {"value": oks / dts, "unit": "solves/s", "ms_per_step": 1000.0 * dts,
         "selector": "learned" if have_sel else "none (AUTO = FP32 + IR)",
         "workers": args.workers, "rungs_used": rungss},
        "workers_ladder": None if args.no_workers else
        {"value": okl / dtl, "unit": "solves/s", "ms_per_step": 1000.0 * dtl,
         "ladder": "fp32 classical IR, then GMRES-IR, then fp64", "rungs_used": rungsl},
        "workers_fp64_direct": None if args.no_workers else
        {"value": okw / dtw, "unit": "solves/s", "ms_per_step": 1000.0 * dtw},
        "roofline": roof,
        "generation_s": gen_s,
    }
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline_batch(probs, args.cpu_seconds)
    return line


GLS_WORKLOAD = ("single GLS d = Wx + Vy: W 4096x1024 N(0,1), V 4096x4096 = U diag(s) V^T "
                "(s log-spaced 1..1e-6), d N(0,1), seed 3")
LSE_WIDE_WORKLOAD = ("single LSE with n > m: A 2048x4096 = U diag(s) V^T (s log-spaced 1..1e-4), "
                     "B 2560x4096 N(0,1), b,d N(0,1), seed 7")
GLS_TALL_WORKLOAD = ("single GLS with n > p: W 4096x2560 N(0,1), V 4096x2048 = U diag(s) V^T "
                     "(s log-spaced 1..1e-4), d N(0,1), seed 8")


def single_gmres(args):
    """One large instance solved by low-precision factorization + GMRES-IR
    (block-diagonal split preconditioner) against the FP64 direct path; a
    solve counts only if it certifies berr <= 1e-14.  gls-large: the GLS with
    n <= p (eq. gls-bdpre-plarge); lse-wide: LSE with n > m
    (eq. lse-bdpre-nlarge); gls-tall: GLS with n > p (eq. gls-bdpre-nlarge)."""
    import torch
    from paper_2406_16499_amd import lsq
    from paper_2406_16499_amd import workloads as wl
    kind = args.workload
    h = lsq.Handle(load_selector=False)
    if kind == "lse-wide":
        prob = wl.lse_conditioned(np.random.default_rng(7), 2048, 4096, 2560, 1e4)
        m, n, p = prob.shape
        A, B, b, d = (lsq.colmajor(a) for a in (prob.A, prob.B, prob.b, prob.d))
        x, r, v = lsq.empty(n), lsq.empty(m), lsq.empty(p)
        solve = lambda opts: h.lse_solve(A, B, b, d, x, r, v, opts)
        workload, shape = LSE_WIDE_WORKLOAD, {"m": m, "n": n, "p": p}
    else:
        if kind == "gls-tall":
            prob = wl.gls_conditioned(np.random.default_rng(8), 4096, 2560, 2048, 1e4)
            workload = GLS_TALL_WORKLOAD
        else:
            prob = wl.config3()
            workload = GLS_WORKLOAD
        n, m, p = prob.shape
        W, V, d = (lsq.colmajor(a) for a in (prob.W, prob.V, prob.d))
        x, y, z = lsq.empty(m), lsq.empty(p), lsq.empty(n)
        solve = lambda opts: h.gls_solve(W, V, d, x, y, z, opts)
        shape = {"n": n, "m": m, "p": p}
    torch.cuda.synchronize()

    def run(opts):
        for _ in range(args.warmup):
            solve(opts)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ok, last = 0, None
        for _ in range(args.steps):
            rc, res = solve(opts)
            last = res.as_dict()
            ok += int(rc == 0 and res.berr_max <= 1e-14)
        torch.cuda.synchronize()
        return time.perf_counter() - t0, ok, last

    prec = args.prec if args.prec in ("bf16", "fp16", "fp32") else "fp16"
    dt, ok, last = run(lsq.default_opts(prec=prec, solver="gmres", escalate=1))
    dt64, ok64, last64 = run(lsq.default_opts(prec="fp64", solver="direct"))
    value, value64 = ok / dt, ok64 / dt64
    h.close()
    return ({
        "metric": METRIC, "value": value, "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1000.0 * dt / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": f"f64 (residuals, GMRES) / {prec} (factorization)", "data": "synthetic",
        "config": {"workload": workload, **shape, "factorization": prec,
                   "solver": "GMRES-IR, block-diagonal split preconditioner, restart 30",
                   "tol": 1e-14},
        "fp64_direct": {"value": value64, "unit": "solves/s", "ms_per_step": 1000.0 * dt64 / args.steps,
                        "last_result": last64},
        "speedup_vs_fp64": value / value64 if value64 > 0 else None,
        "certified_solves": ok, "last_result": last})


PAPER_GRID_WORKLOAD = ("the paper's experiment grid (Section 6): E1 LSE m > n >> p, n in {1024, 2048, 3072}, "
                       "(m, p) in {8n, 10n, 12n} x {n/32, n/64}, kappa([A^T, B^T]) in {1e3, 1e5, 1e7, 1e9}; "
                       "E2 LSE m >> n > p, n in {128, 192, 256}, (m, p) in {128n, 256n} x {n/8, n/4, n/2}, "
                       "kappa 1e5; E3 GLS, n in {1024, 2048, 3072}, (p, m) in {8n, 10n, 12n} x "
                       "{n/32, n/64}, kappa([W, V]) in {1e3, 1e5, 1e7, 1e9}; [A^T, B^T] resp. [W, V] = "
                       "U diag(s) V^T with Haar U, V and log-spaced s; RHS N(0,1); seed 11")


def grid_cases(exps, ns):
    """Groups (n, big, small, [(exp, kind, kappas), ...]) of the paper's grid:
    E1's (m, p) = (big, small) and E3's (p, m) = (big, small) share the shape
    of the stacked matrix, so one pair of orthogonal bases serves both and
    every kappa."""
    groups = []
    if "E1" in exps or "E3" in exps:
        for n in [x for x in (1024, 2048, 3072) if not ns or x in ns]:
            for fm in (8, 10, 12):
                for fp in (32, 64):
                    runs = [(e, "lse" if e == "E1" else "gls", (1e3, 1e5, 1e7, 1e9))
                            for e in ("E1", "E3") if e in exps]
                    groups.append((n, fm * n, n // fp, runs))
    if "E2" in exps:
        for n in [x for x in (128, 192, 256) if not ns or x in ns]:
            for fm in (128, 256):
                for fp in (8, 4, 2):
                    groups.append((n, fm * n, n // fp, [("E2", "lse", (1e5,))]))
    return groups


def paper_grid(args):
    """The paper's experiment grid on the GPU: for every case, the FP32
    factorization with classical IR and with GMRES-IR (escalation on) against
    the FP64 direct path, with the time, refinement steps, backward error and
    the err-1 / err-2 measures of Tables 4 (LSE) and 5 (GLS), err-2 taken
    against the FP64 direct solution."""
    import torch
    from paper_2406_16499_amd import lsq
    from paper_2406_16499_amd import workloads as wl
    h = lsq.Handle(load_selector=False)
    exps = [e for e in args.grid.split(",") if e]
    ns = [int(x) for x in args.grid_n.split(",") if x] if args.grid_n else []
    rng = np.random.default_rng(11)
    nrm = np.linalg.norm
    rows = []
    t_mixed = t_fp64 = 0.0
    ok_mixed = ok_fp64 = 0
    for (n, big, small, runs) in grid_cases(exps, ns):
        N = big + small
        U, Vb = wl.paper_bases(rng, n, N)
        for (exp, kind, kappa) in [(e, k, kp) for (e, k, kps) in runs for kp in kps]:
            if kind == "lse":
                m, p = big, small
                P = wl.lse_paper_from_bases(rng, U, Vb, m, p, kappa)
                A, B, b, d = (lsq.colmajor(a) for a in (P.A, P.B, P.b, P.d))
                x, r, v = lsq.empty(n), lsq.empty(m), lsq.empty(p)
                solve = lambda o: h.lse_solve(A, B, b, d, x, r, v, o)
                sol = lambda: x.detach().cpu().numpy().copy()
                fro_b = nrm(P.B)
                err1 = lambda xs: float(nrm(P.B @ xs - P.d) / (fro_b * nrm(xs) + nrm(P.d)))
                res_ref = {}
                def err2(xs, xr):
                    if "r" not in res_ref:
                        res_ref["r"] = nrm(P.A @ xr - P.b)
                    return float(abs(nrm(P.A @ xs - P.b) / res_ref["r"] - 1.0))
                shape = {"m": m, "n": n, "p": p}
            else:
                p, m = big, small
                G = wl.gls_paper_from_bases(rng, U, Vb, m, p, kappa)
                W, V, d = (lsq.colmajor(a) for a in (G.W, G.V, G.d))
                x, y, z = lsq.empty(m), lsq.empty(p), lsq.empty(n)
                solve = lambda o: h.gls_solve(W, V, d, x, y, z, o)
                sol = lambda: (x.detach().cpu().numpy().copy(), y.detach().cpu().numpy().copy())
                fw, fv = nrm(G.W), nrm(G.V)
                err1 = lambda s_: float(nrm(G.W @ s_[0] + G.V @ s_[1] - G.d)
                                        / (fw * nrm(s_[0]) + fv * nrm(s_[1]) + nrm(G.d)))
                err2 = lambda s_, sr: float(abs(nrm(s_[1]) / nrm(sr[1]) - 1.0))
                shape = {"n": n, "m": m, "p": p}
            torch.cuda.synchronize()
            out = {"exp": exp, "kind": kind, **shape, "kappa": kappa}
            ref = None
            for name, opts in (("fp64", lsq.default_opts(prec="fp64", solver="direct")),
                               ("ir", lsq.default_opts(prec="fp32", solver="ir", escalate=1)),
                               ("gmres", lsq.default_opts(prec="fp32", solver="gmres", escalate=1))):
                for _ in range(args.warmup):
                    solve(opts)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                ok = 0
                for _ in range(args.steps):
                    rc, res = solve(opts)
                    ok += int(rc == 0 and res.berr_max <= 1e-14)
                torch.cuda.synchronize()
                dt = (time.perf_counter() - t0) / args.steps
                dd = res.as_dict()
                xs = sol()
                if name == "fp64":
                    ref = xs
                out[name] = {"ms": 1000.0 * dt, "certified": ok, "steps": args.steps,
                             "rung": f"{dd['prec_used']}/{dd['solver_used']}", "attempts": dd["attempts"],
                             "ir_steps": dd["ir_steps"], "gmres_iters": dd["gmres_iters"],
                             "berr": dd["berr_max"], "err1": err1(xs), "err2": err2(xs, ref)}
            t_fp64 += out["fp64"]["ms"]
            ok_fp64 += out["fp64"]["certified"]
            best = min((out["ir"], out["gmres"]), key=lambda e: e["ms"])
            t_mixed += best["ms"]
            ok_mixed += best["certified"]
            out["time_ratio_best_mixed_vs_fp64"] = best["ms"] / out["fp64"]["ms"]
            rows.append(out)
            print(f"[grid] {exp} {kind} {shape} kappa={kappa:g} fp64 {out['fp64']['ms']:.1f} ms, "
                  f"ir {out['ir']['ms']:.1f} ms ({out['ir']['rung']}, {out['ir']['ir_steps']} steps, "
                  f"err1 {out['ir']['err1']:.1e} err2 {out['ir']['err2']:.1e}), gmres {out['gmres']['ms']:.1f} ms "
                  f"({out['gmres']['rung']}, {out['gmres']['gmres_iters']} it)", file=sys.stderr, flush=True)
            del solve, sol
        del U, Vb
    ncase = len(rows)
    value = 1000.0 * ncase / t_mixed if t_mixed > 0 else 0.0
    print(json.dumps({
        "metric": METRIC, "value": value, "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": t_mixed, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64 (residuals, updates) / fp32 (factorization)",
        "data": "synthetic",
        "config": {"workload": PAPER_GRID_WORKLOAD, "experiments": exps, "n": ns or "all",
                   "cases": ncase,
                   "solver": "per case the faster of classical IR and GMRES-IR (FP32 factors, escalation on)",
                   "tol": 1e-14},
        "fp64_direct": {"value": 1000.0 * ncase / t_fp64 if t_fp64 > 0 else 0.0, "unit": "solves/s",
                        "ms_per_step": t_fp64},
        "speedup_vs_fp64": t_fp64 / t_mixed if t_mixed > 0 else None,
        "certified_mixed": ok_mixed, "certified_fp64": ok_fp64, "cases": rows}))


def lse_factored(args):
    """The default large LSE factored once (FP32), then solves with a fresh
    right-hand side (b, d) each step: refinement only, against full solves of
    the same right-hand sides."""
    import torch
    from paper_2406_16499_amd import lsq
    from paper_2406_16499_amd import workloads as wl
    prob = wl.config2()
    m, n, p = prob.shape
    rng = np.random.default_rng(12)
    A, B = lsq.colmajor(prob.A), lsq.colmajor(prob.B)
    rhs = [(lsq.colmajor(rng.standard_normal(m)), lsq.colmajor(rng.standard_normal(p)))
           for _ in range(args.steps + args.warmup)]
    x, r, v = lsq.empty(n), lsq.empty(m), lsq.empty(p)
    h = lsq.Handle(load_selector=False)
    o = lsq.default_opts(prec="fp32", solver="ir", escalate=0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    F = h.lse_factor(A, B, "fp32")
    torch.cuda.synchronize()
    t_factor = time.perf_counter() - t0

    def run(solve):
        for j in range(args.warmup):
            solve(*rhs[j])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ok = 0
        for j in range(args.warmup, args.warmup + args.steps):
            rc, res = solve(*rhs[j])
            ok += int(rc == 0 and res.berr_max <= 1e-14)
        torch.cuda.synchronize()
        return time.perf_counter() - t0, ok, res.as_dict()

    dt, ok, last = run(lambda b, d: F.solve(b, d, x, r, v, opts=o))
    dtf, okf, lastf = run(lambda b, d: h.lse_solve(A, B, b, d, x, r, v, o))
    F.close()
    print(json.dumps({
        "metric": METRIC, "value": ok / dt, "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1000.0 * dt / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "f64 (residuals, updates) / fp32 (stored factors)", "data": "synthetic",
        "config": {"workload": WORKLOAD + "; factored once, a new (b, d) per step", "m": m, "n": n,
                   "p": p, "factorization": "fp32", "solver": "classical IR on stored factors",
                   "tol": 1e-14},
        "factor_ms": 1000.0 * t_factor,
        "full_solve": {"value": okf / dtf, "unit": "solves/s", "ms_per_step": 1000.0 * dtf / args.steps},
        "certified_solves": ok, "last_result": last}))


def roofline_of(timing, kernel, steps, files=None):
    """Roofline object of one timed kernel kind: achieved = algorithmic work per
    launch / average event-timed launch duration."""
    if timing is None or timing[1] <= 0:
        return None
    total_ms, launches, flops, nbytes = timing
    name, bound, peak, unit = KERNELS[kernel]
    avg_s = total_ms * 1e-3 / launches
    achieved = (nbytes / launches / avg_s / 1e9) if bound == "hbm" else (flops / launches / avg_s / 1e12)
    return {"bound": bound, "achieved": achieved, "peak": peak, "unit": unit, "frac": achieved / peak,
            "traffic": traffic_per_launch(kernel, files), "kernel": name,
            "launches_per_step": launches / steps, "avg_launch_us": avg_s * 1e6,
            "alg_flops_per_launch": flops / launches, "alg_bytes_per_launch": nbytes / launches,
            "source_hash": source_hash(files)}


def lse_large(args, cpu=True):
    """The single large LSE: FP32 (and BF16) factorization with classical IR and
    the escalation ladder against the FP64 direct path."""
    import torch
    from paper_2406_16499_amd import lsq
    from paper_2406_16499_amd import workloads as wl

    prob = wl.config2(m=args.m, n=args.n, p=args.p)
    tensors = tuple(lsq.colmajor(a) for a in (prob.A, prob.B, prob.b, prob.d))
    torch.cuda.synchronize()
    h = lsq.Handle()
    precs = [args.prec] + (["bf16"] if args.prec == "fp32" else [])
    mixed = {}
    for prec in precs:
        o = lsq.default_opts(prec=prec, solver="ir", escalate=1)
        mixed[prec] = time_solves(h, lsq, torch, tensors, o, args.steps, args.warmup,
                                  kernel=args.kernel if prec == args.prec else None)
    fp64_opts = lsq.default_opts(prec="fp64", solver="direct")
    dt_64, ok_64, res_64, _ = time_solves(h, lsq, torch, tensors, fp64_opts, args.steps, args.warmup)
    # the HBM-bound refinement kernels, timed on extra mixed solves (outside
    # the solves/s figures): the FP64 residual sweep and the reflector GEMVs
    o32 = lsq.default_opts(prec=args.prec, solver="ir", escalate=1)
    hbm = {}
    for k in ("dual_gemv", "agg_gemv"):
        _, _, _, tk = time_solves(h, lsq, torch, tensors, o32, 2, 0, kernel=k)
        hbm[k] = roofline_of(tk, k, 2)
    # calibration copy of known size, outside the timed regions (scales the
    # FETCH_SIZE / WRITE_SIZE counters of a profiled run)
    src = torch.empty(COPY_BYTES // 8, dtype=torch.float64, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    h.dbg_copy(dst, src, COPY_BYTES)
    del src, dst
    h.close()

    dt_mix, ok_mix, res_mix, timing = mixed[args.prec]
    value = ok_mix / dt_mix
    value64 = ok_64 / dt_64
    m, n, p = args.m, args.n, args.p
    # algorithmic work of one generalized RQ (Section 3.1 flop model, leading terms):
    # RQ of B 2np^2 - 2p^3/3, A Q^T 4mnp - 2mp^2, QR of A Q^T 2mn^2 - 2n^3/3
    tf = (2 * n * p * p - 2 * p ** 3 / 3) + (4 * m * n * p - 2 * m * p * p) + (2 * m * n * n - 2 * n ** 3 / 3)
    line = {
        "metric": METRIC, "value": value, "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1000.0 * dt_mix / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "f64 (residuals, updates) / " + args.prec + " (factorization)", "data": "synthetic",
        "config": {"workload": WORKLOAD, "m": m, "n": n, "p": p, "factorization": args.prec,
                   "solver": "classical IR with escalation ladder", "tol": 1e-14},
        "fp64_direct": {"value": value64, "unit": "solves/s", "ms_per_step": 1000.0 * dt_64 / args.steps,
                        "certified": ok_64},
        "speedup_vs_fp64": value / value64 if value64 > 0 else None,
        "certified_solves": ok_mix,
        "last_result": res_mix[-1] if res_mix else None,
        "last_result_fp64": res_64[-1] if res_64 else None,
        "factor_flops": tf,
        "factor_tflops": {"mixed": tf / (res_mix[-1]["ms_factor"] * 1e-3) / 1e12 if res_mix else None,
                          "fp64": tf / (res_64[-1]["ms_factor"] * 1e-3) / 1e12 if res_64 else None},
        "roofline": roofline_of(timing, args.kernel, args.steps),
        "hbm_kernels": hbm,
    }
    for prec in precs[1:]:
        dt, ok, res, _ = mixed[prec]
        line[f"mixed_{prec}"] = {"value": ok / dt, "unit": "solves/s", "ms_per_step": 1000.0 * dt / args.steps,
                                 "speedup_vs_fp64": (ok / dt) / value64 if value64 > 0 else None,
                                 "certified": ok, "last_result": res[-1] if res else None}
    if cpu and not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(prob, args.cpu_seconds)
    return line


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: the solver runs on one GPU; --gpus {args.gpus} is not supported "
              "(a multi-GPU run would shard the batched instances across GPUs)",
              file=sys.stderr)
        sys.exit(2)
    if args.workload == "batched":
        print(json.dumps(batched(args)))
        return
    if args.workload in ("gls-large", "lse-wide", "gls-tall"):
        print(json.dumps(single_gmres(args)))
        return
    if args.workload == "paper-grid":
        return paper_grid(args)
    if args.workload == "lse-factored":
        return lse_factored(args)
    if args.workload == "lse-large":
        print(json.dumps(lse_large(args)))
        return
    # headline: the batched workload, with the large LSE and GLS as sub-records
    line = batched(args)
    print("[bench] batched done", file=sys.stderr, flush=True)
    regimes = {f"batched_kappa_{k:.0e}".replace("+0", ""): batched_regime(args, k) for k in (1e3, 1e5)}
    print("[bench] conditioning regimes done", file=sys.stderr, flush=True)
    sub_lse = lse_large(args, cpu=False)
    print("[bench] large LSE done", file=sys.stderr, flush=True)
    gls_args = argparse.Namespace(**vars(args))
    gls_args.workload, gls_args.prec = "gls-large", "fp16"
    gls_args.steps, gls_args.warmup = min(args.steps, 3), min(args.warmup, 1)
    sub_gls = single_gmres(gls_args)
    print("[bench] large GLS done", file=sys.stderr, flush=True)
    keep = ("value", "unit", "ms_per_step", "steps", "config", "fp64_direct", "speedup_vs_fp64",
            "certified_solves", "last_result", "last_result_fp64", "factor_flops", "factor_tflops",
            "roofline", "hbm_kernels", "mixed_bf16")
    line["sub_records"] = {
        "lse_large": {k: sub_lse[k] for k in keep if k in sub_lse},
        "gls_large": {k: sub_gls[k] for k in keep if k in sub_gls},
        **regimes,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
