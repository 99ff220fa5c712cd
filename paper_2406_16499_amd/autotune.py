"""Autotuner of the persistent batch's launch shape.

The persistent batched solver (liblsq: lsq_solve_batched, persistent modes)
runs an FP32 launch and, beside it, FP64 work-groups that take the instances
the FP32 rung does not certify.  Three run-time parameters shape it: the
share of compute units the FP64 rung starts on, the diagonal-ratio route that
sends an instance on to FP64 without refining, and the number of the longest
instances (per FP64 work-group) that go to FP64 from the start.  Their best
values depend on the instance sizes and on how many instances escalate.  The
tuner measures every point of a grid on batches of the recipe of
workloads.batch_instances restricted to one size bucket at a time, for two
conditioning regimes (both condition numbers up to 1e8, where a large share
escalates, and up to 1e5, where almost none does), keeps the fastest point
that certifies every instance per bucket and regime, and writes the table to
batch_tuning.json beside this file; Handle() installs it (lsq_batch_tuning).
An entry of the well-conditioned regime applies while the handle's last
FP32-first batch escalated at most the midpoint of the fractions the two
regimes showed under their chosen points.

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
# conditioning regimes: (kappa_max of the recipe, routes, shares, pres)
REGIMES = [
    (1e8, [1e5, 3e5], [0.4375, 0.5, 0.5625, 0.625], [3.0, 4.0, 6.0, 8.0]),
    (1e5, [3e5], [0.03125, 0.0625, 0.125, 0.1875], [0.0, 1.0, 2.0, 4.0]),
]


def load(path: str = TUNING_PATH):
    """[(max_dim, route, fp64_share, pre, esc_max)] from the stored table, or []."""
    if not os.path.exists(path):
        return []
    with open(path) as fh:
        doc = json.load(fh)
    return [(int(e["max_dim"]), float(e["route"]), float(e["fp64_share"]), float(e.get("pre", 0.0)),
             float(e.get("esc_max", 1.0)))
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
        chosen = []
        for kappa_max, routes, shares, pres in REGIMES:
            probs = list(wl.batch_instances(seed=seed, count=count, kappa_max=kappa_max, m_range=(lo, hi)))
            ups = [_device_problem(P) for P in probs]
            descs = [d for d, _ in ups]
            torch.cuda.synchronize()
            # keep the interpreter's full collections (a pause of tens of ms
            # over thousands of tensors) out of the timed calls
            gc.collect()
            gc.freeze()
            rows = []
            for route in routes:
                for share in shares:
                    for pre in pres:
                        h.dbg_batch_route(route)
                        h.dbg_batch_split(share)
                        h.dbg_batch_pre(pre)
                        rate, worst, frac = measure(h, descs, opts, steps)
                        rows.append({"route": route, "fp64_share": share, "pre": pre, "solves_per_s": rate,
                                     "slowest_call_solves_per_s": worst, "certified": frac})
                        log(f"  m <= {hi}, kappa <= {kappa_max:g}: route {route:g} share {share:g} pre {pre:g}: "
                            f"{rate:,.0f} solves/s (slowest call {worst:,.0f}), {frac:.4f} certified")
            good = [r for r in rows if r["certified"] == 1.0] or rows
            best = max(good, key=lambda r: r["solves_per_s"])
            # the escalation fraction this regime shows under its chosen point
            h.dbg_batch_route(best["route"])
            h.dbg_batch_split(best["fp64_share"])
            h.dbg_batch_pre(best["pre"])
            h.lsq_solve_batched(descs, opts)
            esc = h.dbg_batch_regime()
            chosen.append((kappa_max, best, esc))
            grids.append({"max_dim": hi, "kappa_max": kappa_max, "escalation": esc, "grid": rows})
            log(f"bucket m <= {hi}, kappa <= {kappa_max:g}: route {best['route']:g}, share "
                f"{best['fp64_share']:g}, pre {best['pre']:g}, escalation {esc:.4f}")
            gc.unfreeze()
            del ups, descs, probs
            gc.collect()
        (_, ill, esc_ill), (_, well, esc_well) = chosen
        threshold = 0.5 * (esc_ill + esc_well)
        entries.append({"max_dim": hi, "route": ill["route"], "fp64_share": ill["fp64_share"], "pre": ill["pre"],
                        "esc_max": 1.0, "solves_per_s": ill["solves_per_s"]})
        if esc_well < esc_ill:
            entries.append({"max_dim": hi, "route": well["route"], "fp64_share": well["fp64_share"],
                            "pre": well["pre"], "esc_max": threshold, "solves_per_s": well["solves_per_s"]})
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
    doc = {"workload": f"batch recipe, {a.count} instances per bucket and regime, seed {a.seed}, "
                       f"kappa <= {', '.join(f'{r[0]:g}' for r in REGIMES)}",
           "entries": entries, "grids": grids}
    with open(a.out, "w") as fh:
        json.dump(doc, fh, indent=1)
    print(json.dumps({"entries": entries}))


if __name__ == "__main__":
    main()
