"""Benchmark: LSE solves/s at FP64 backward error <= 1e-14, mixed-precision
refinement vs the all-FP64 GPU path, on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--prec fp32] [--no-cpu]

Workload: single large LSE, A 4096 x 2048 = U diag(s) V^T (Haar U, V; s
log-spaced 1 .. 1e-4, kappa(A) = 1e4), B 256 x 2048 i.i.d. N(0,1), b, d
i.i.d. N(0,1) (seed 2), synthetic and resident in HBM before timing starts.
A step is one complete solve through the C-ABI: down-conversion, generalized
RQ factorization at u_f, initial guess, and refinement until the stopping
test (eq. lse-stop, tol = 1e-14) holds; a solve that does not certify
berr <= 1e-14 is not counted.

Prints one JSON line (rank 0 only; the solver runs on one GPU).
"""
from __future__ import annotations

import argparse
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
PEAK_FP32_VECTOR = 157.3                                              # TFLOP/s
COPY_BYTES = 256 << 20            # calibration copy for the hardware byte counters
# Kernel whose roofline is reported, with its bound: the Householder panel
# reconstruction dominates the mixed-precision solve (FP64 arithmetic).
KERNELS = {
    "panel_final_y": ("k_panel_final_y", "mfma", 78.6, "TFLOP/s"),
    "panel_cholpass": ("k_panel_cholpass", "mfma", 78.6, "TFLOP/s"),
    "wy_u": ("k_wy_u", "mfma", None, "TFLOP/s"),
    "wy_t": ("k_wy_t", "mfma", None, "TFLOP/s"),
    "dual_gemv": ("k_dual_gemv", "hbm", HBM_PEAK, "GB/s"),
}
KERNEL_SOURCES = ["paper_2406_16499_amd/csrc/qr.hip", "paper_2406_16499_amd/csrc/wg64.hpp",
                  "paper_2406_16499_amd/csrc/vec.hip", "paper_2406_16499_amd/csrc/common.hpp",
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
    ap.add_argument("--workload", default="lse-large",
                    choices=["lse-large", "gls-large", "lse-wide", "gls-tall", "paper-grid", "lse-factored",
                             "batched"],
                    help="lse-large: the single 4096x2048x256 LSE (default); gls-large: the "
                         "4096x1024x4096 GLS with GMRES-IR; lse-wide: LSE 2048x4096x2560 (n > m) "
                         "with GMRES-IR; gls-tall: GLS 4096x2560x2048 (n > p) with GMRES-IR; "
                         "paper-grid: the paper's experiment shapes against the GPU FP64 path; "
                         "lse-factored: the default LSE factored once, solves with new right-hand sides; "
                         "batched: the 2000-instance mixed LSE/GLS workload")
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
    h = lsq.Handle()
    h.lib.lsq_set_batch_workers(h.h, args.workers)

    def run(opts, steps, warmup, mode="persistent", kernel=None):
        h.set_batch_mode(mode)
        for _ in range(warmup):
            h.lsq_solve_batched(descs, opts)
        torch.cuda.synchronize()
        if kernel:
            h.timer_enable(kernel)
        t1 = time.perf_counter()
        ok, rungs = 0, {}
        for _ in range(steps):
            rc, res = h.lsq_solve_batched(descs, opts)
            for r in res:
                if r.info == 0 and r.berr_max <= 1e-14:
                    ok += 1
                d = r.as_dict()
                key = f"{d['prec_used']}/{d['solver_used']}"
                rungs[key] = rungs.get(key, 0) + 1
        torch.cuda.synchronize()
        dt = time.perf_counter() - t1
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
    dt, ok, rungs, tim = run(mixed, args.steps, args.warmup, kernel="batch_fp32")
    dt64, ok64, _, tim64 = run(lsq.default_opts(prec="fp64", solver="direct"), args.steps,
                               args.warmup, kernel="batch_fp64")
    # per-instance solves on the batch workers (context): the learned selector
    # picks each instance's starting rung
    auto = lsq.default_opts(prec="auto", solver="auto", escalate=1)
    if not args.no_workers:
        dts, oks, rungss, _ = run(auto, 1, 0, mode="workers")
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
        roof = {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_VECTOR, "unit": "TFLOP/s",
                "frac": achieved / PEAK_FP32_VECTOR,
                "traffic": traffic_per_launch("batch_fp32", BATCH_SOURCES), "kernel": "k_batch<float>",
                "launches_per_step": launches / args.steps, "avg_launch_us": 1000.0 * ms / launches,
                "alg_flops_per_launch": flops / launches,
                "flops_counted": "Householder flops of the factorizations of the instances in the launch",
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
        "certified_fraction": ok / (args.count * args.steps),
        "rungs_used": rungs,
        "workers_selector": None if args.no_workers else
        {"value": oks / dts, "unit": "solves/s", "ms_per_step": 1000.0 * dts,
         "selector": "learned" if have_sel else "none (AUTO = FP32 + IR)",
         "workers": args.workers, "rungs_used": rungss},
        "workers_fp64_direct": None if args.no_workers else
        {"value": okw / dtw, "unit": "solves/s", "ms_per_step": 1000.0 * dtw},
        "roofline": roof,
        "generation_s": gen_s,
    }
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline_batch(probs, args.cpu_seconds)
    print(json.dumps(line))


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
    print(json.dumps({
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
        "certified_solves": ok, "last_result": last}))


PAPER_GRID_WORKLOAD = ("the paper's experiment shapes (Section 6): LSE m > n >> p (n 1024, (m, p) = "
                       "(8n, n/32), (12n, n/64)) and m >> n > p (n 128, (m, p) = (128n, n/8)); GLS "
                       "(n 1024, (p, m) = (8n, n/32), (12n, n/64)); [A^T, B^T] resp. [W, V] = "
                       "U diag(s) V^T with log-spaced s, kappa 1e3..1e9; RHS N(0,1); seed 11")


def paper_grid(args):
    """The paper's experiment shapes on the GPU: for every case, the FP32
    factorization with classical IR and with GMRES-IR (escalation on), and the
    FP64 direct path; times, refinement steps, backward errors and the
    distance of the mixed solution from the FP64 one (the relative-time and
    error columns of Tables 4 and 5, against the GPU FP64 path)."""
    import torch
    from paper_2406_16499_amd import lsq
    from paper_2406_16499_amd import workloads as wl
    h = lsq.Handle(load_selector=False)
    rng = np.random.default_rng(11)
    cases = []
    for kappa in (1e3, 1e5, 1e7, 1e9):
        for (fm, fp) in ((8, 32), (12, 64)):
            cases.append(("E1", "lse", 1024, fm, fp, kappa))
    cases.append(("E2", "lse", 128, 128, 8, 1e5))
    for kappa in (1e3, 1e5, 1e7, 1e9):
        for (fm, fp) in ((8, 32), (12, 64)):
            cases.append(("E3", "gls", 1024, fm, fp, kappa))
    rows = []
    t_mixed = t_fp64 = 0.0
    ok_mixed = ok_fp64 = 0
    for (exp, kind, n, fm, fp, kappa) in cases:
        if kind == "lse":
            m, p = fm * n, n // fp
            P = wl.lse_paper_pair(rng, m, n, p, kappa)
            A, B, b, d = (lsq.colmajor(a) for a in (P.A, P.B, P.b, P.d))
            x, r, v = lsq.empty(n), lsq.empty(m), lsq.empty(p)
            solve = lambda o: h.lse_solve(A, B, b, d, x, r, v, o)
            sol = lambda: x.detach().cpu().numpy().copy()
            shape = {"m": m, "n": n, "p": p}
        else:
            p_, m_ = fm * n, n // fp
            G = wl.gls_paper_pair(rng, n, m_, p_, kappa)
            W, V, d = (lsq.colmajor(a) for a in (G.W, G.V, G.d))
            x, y, z = lsq.empty(m_), lsq.empty(p_), lsq.empty(n)
            solve = lambda o: h.gls_solve(W, V, d, x, y, z, o)
            sol = lambda: np.concatenate([x.detach().cpu().numpy(), y.detach().cpu().numpy()])
            shape = {"n": n, "m": m_, "p": p_}
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
            den = float(np.max(np.abs(ref))) if ref is not None and ref.size else 0.0
            dist = float(np.max(np.abs(xs - ref)) / den) if den > 0 else 0.0
            out[name] = {"ms": 1000.0 * dt, "certified": ok, "steps": args.steps,
                         "rung": f"{dd['prec_used']}/{dd['solver_used']}", "attempts": dd["attempts"],
                         "ir_steps": dd["ir_steps"], "gmres_iters": dd["gmres_iters"],
                         "berr": dd["berr_max"], "dist_to_fp64": dist}
        t_fp64 += out["fp64"]["ms"]
        ok_fp64 += out["fp64"]["certified"]
        best = min((out["ir"], out["gmres"]), key=lambda e: e["ms"])
        t_mixed += best["ms"]
        ok_mixed += best["certified"]
        out["time_ratio_best_mixed_vs_fp64"] = best["ms"] / out["fp64"]["ms"]
        rows.append(out)
        print(f"[grid] {exp} {kind} {shape} kappa={kappa:g} fp64 {out['fp64']['ms']:.1f} ms, "
              f"ir {out['ir']['ms']:.1f} ms ({out['ir']['rung']}), gmres {out['gmres']['ms']:.1f} ms "
              f"({out['gmres']['rung']})", file=sys.stderr, flush=True)
    ncase = len(rows)
    value = 1000.0 * ncase / t_mixed if t_mixed > 0 else 0.0
    print(json.dumps({
        "metric": METRIC, "value": value, "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": t_mixed, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64 (residuals, updates) / fp32 (factorization)",
        "data": "synthetic",
        "config": {"workload": PAPER_GRID_WORKLOAD, "cases": ncase,
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


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: the solver runs on one GPU; --gpus {args.gpus} is not supported "
              "(a multi-GPU run would shard the batched instances across GPUs)",
              file=sys.stderr)
        sys.exit(2)
    if args.workload == "batched":
        return batched(args)
    if args.workload in ("gls-large", "lse-wide", "gls-tall"):
        return single_gmres(args)
    if args.workload == "paper-grid":
        return paper_grid(args)
    if args.workload == "lse-factored":
        return lse_factored(args)
    import torch
    from paper_2406_16499_amd import lsq
    from paper_2406_16499_amd import workloads as wl

    prob = wl.config2(m=args.m, n=args.n, p=args.p)
    tensors = tuple(lsq.colmajor(a) for a in (prob.A, prob.B, prob.b, prob.d))
    torch.cuda.synchronize()
    h = lsq.Handle()

    mixed_opts = lsq.default_opts(prec=args.prec, solver="ir", escalate=1)
    fp64_opts = lsq.default_opts(prec="fp64", solver="direct")
    dt_mix, ok_mix, res_mix, timing = time_solves(h, lsq, torch, tensors, mixed_opts, args.steps,
                                                  args.warmup, kernel=args.kernel)
    dt_64, ok_64, res_64, _ = time_solves(h, lsq, torch, tensors, fp64_opts, args.steps, args.warmup)
    # calibration copy of known size, outside the timed regions (scales the
    # FETCH_SIZE / WRITE_SIZE counters of a profiled run)
    src = torch.empty(COPY_BYTES // 8, dtype=torch.float64, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    h.dbg_copy(dst, src, COPY_BYTES)
    del src, dst

    value = ok_mix / dt_mix
    value64 = ok_64 / dt_64
    m, n, p = args.m, args.n, args.p
    # algorithmic work of one generalized RQ (Section 3.1 flop model, leading terms):
    # RQ of B 2np^2 - 2p^3/3, A Q^T 4mnp - 2mp^2, QR of A Q^T 2mn^2 - 2n^3/3
    tf = (2 * n * p * p - 2 * p ** 3 / 3) + (4 * m * n * p - 2 * m * p * p) + (2 * m * n * n - 2 * n ** 3 / 3)

    roof = None
    if timing is not None and timing[1] > 0:
        total_ms, launches, flops, nbytes = timing
        name, bound, peak, unit = KERNELS[args.kernel]
        if peak is None:
            peak = PEAK.get(args.prec, PEAK["fp32"])
        avg_s = total_ms * 1e-3 / launches
        if bound == "hbm":
            achieved = nbytes / launches / avg_s / 1e9
        else:
            achieved = flops / launches / avg_s / 1e12
        traffic = traffic_per_launch(args.kernel)
        roof = {"bound": bound, "achieved": achieved, "peak": peak, "unit": unit,
                "frac": achieved / peak, "traffic": traffic,
                "kernel": name, "launches_per_step": launches / args.steps,
                "avg_launch_us": avg_s * 1e6,
                "alg_flops_per_launch": flops / launches, "alg_bytes_per_launch": nbytes / launches,
                "source_hash": source_hash()}

    line = {
        "metric": METRIC,
        "value": value,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1000.0 * dt_mix / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64 (residuals, updates) / " + args.prec + " (factorization)",
        "data": "synthetic",
        "config": {"workload": WORKLOAD, "m": m, "n": n, "p": p, "factorization": args.prec,
                   "solver": "classical IR with escalation ladder", "tol": 1e-14},
        "fp64_direct": {"value": value64, "unit": "solves/s", "ms_per_step": 1000.0 * dt_64 / args.steps,
                        "certified": ok_64},
        "speedup_vs_fp64": value / value64 if value64 > 0 else None,
        "certified_solves": ok_mix,
        "last_result": res_mix[-1] if res_mix else None,
        "last_result_fp64": res_64[-1] if res_64 else None,
        "factor_flops": tf,
        "roofline": roof,
    }
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(prob, args.cpu_seconds)
    print(json.dumps(line))


if __name__ == "__main__":
    main()
