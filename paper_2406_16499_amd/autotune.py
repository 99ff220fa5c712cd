"""Autotuner of the persistent batch's launch shape.

The persistent batched solver (liblsq: lsq_solve_batched, persistent modes)
runs an FP32 launch and, beside it, FP64 work-groups that take the instances
the FP32 rung does not certify.  Three run-time parameters shape it: the
share of compute units the FP64 rung starts on, the diagonal-ratio route that
sends an instance on to FP64 without refining, and the number of the longest
instances (per FP64 work-group) that go to FP64 from the start.  Their best
values depend on the instance sizes.  The tuner measures every point of a
grid on batches of the recipe of workloads.batch_instances restricted to one
size bucket at a time, keeps the fastest point that certifies every instance
per bucket, and writes the table to batch_tuning.json beside this file;
Handle() installs it (lsq_batch_tuning).

    python -m paper_2406_16499_amd.autotune [--count 2000] [--seed 21]
"""
from __future__ import annotations

import argparse
import gc
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
TUNING_PATH = os.path.join(HERE, "batch_tuning.json")
# size buckets: the largest dimension of a batch's instances
BUCKETS = [(64, 256), (64, 512), (64, 1024)]
ROUTES = [1e5, 3e5]
SHARES = [0.4375, 0.5, 0.5625, 0.625]
PRES = [3.0, 4.0, 6.0, 8.0]


def load(path: str = TUNING_PATH):
    """[(max_dim, route, fp64_share, pre)] from the stored table, or []."""
    if not os.path.exists(path):
        return []
    with open(path) as fh:
        doc = json.load(fh)
    return [(int(e["max_dim"]), float(e["route"]), float(e["fp64_share"]), float(e.get("pre", 0.0)))
            for e in doc["entries"]]


def measure(h, descs, opts, steps=5):
    """(solves/s of the median call, of the slowest call, certified
    fraction) of the persistent batch over descs; each call returns only
    once the batch is solved."""
    import statistics
    h.lsq_solve_batched(descs, opts)
    times, ok = [], 0
    for _ in range(steps):
        t0 = time.perf_counter()
        rc, res = h.lsq_solve_batched(descs, opts)
        times.append(time.perf_counter() - t0)
        ok += sum(1 for r in res if rc == 0 and r.info == 0 and r.berr_max <= 1e-14)
    return len(descs) / statistics.median(times), len(descs) / max(times), ok / (len(descs) * steps)


def tune(h, count, seed, log=print, steps=5):
    import torch
    from . import lsq
    from . import workloads as wl
    from .selector import _device_problem
    opts = lsq.default_opts(prec="fp32", solver="ir", escalate=1)
    h.batch_tuning([])
    h.set_batch_mode("persistent")
    entries, grids = [], []
    for lo, hi in BUCKETS:
        probs = list(wl.batch_instances(seed=seed, count=count, kappa_max=1e8, m_range=(lo, hi)))
        ups = [_device_problem(P) for P in probs]
        descs = [d for d, _ in ups]
        torch.cuda.synchronize()
        # keep the interpreter's full collections (a pause of tens of ms over
        # thousands of tensors) out of the timed calls
        gc.collect()
        gc.freeze()
        rows = []
        for route in ROUTES:
            for share in SHARES:
                for pre in PRES:
                    h.dbg_batch_route(route)
                    h.dbg_batch_split(share)
                    h.dbg_batch_pre(pre)
                    rate, worst, frac = measure(h, descs, opts, steps)
                    rows.append({"route": route, "fp64_share": share, "pre": pre, "solves_per_s": rate,
                                 "slowest_call_solves_per_s": worst, "certified": frac})
                    log(f"  m <= {hi}: route {route:g} share {share:g} pre {pre:g}: {rate:,.0f} solves/s "
                        f"(slowest call {worst:,.0f}), {frac:.4f} certified")
        good = [r for r in rows if r["certified"] == 1.0] or rows
        best = max(good, key=lambda r: r["solves_per_s"])
        entries.append({"max_dim": hi, "route": best["route"], "fp64_share": best["fp64_share"],
                        "pre": best["pre"], "solves_per_s": best["solves_per_s"]})
        grids.append({"max_dim": hi, "grid": rows})
        log(f"bucket m <= {hi}: route {best['route']:g}, share {best['fp64_share']:g}, pre {best['pre']:g}")
        del ups, descs
    return entries, grids


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--count", type=int, default=2000)
    ap.add_argument("--seed", type=int, default=21)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--out", default=TUNING_PATH)
    a = ap.parse_args(argv)
    sys.path.insert(0, os.path.dirname(HERE))
    from . import lsq
    h = lsq.Handle(load_selector=False, load_tuning=False)
    log = lambda s: print(s, flush=True)  # noqa: E731
    entries, grids = tune(h, a.count, a.seed, log, a.steps)
    doc = {"workload": f"batch recipe, {a.count} instances per bucket, seed {a.seed}, kappa <= 1e8",
           "entries": entries, "grids": grids}
    with open(a.out, "w") as fh:
        json.dump(doc, fh, indent=1)
    print(json.dumps({"entries": entries}))


if __name__ == "__main__":
    main()
