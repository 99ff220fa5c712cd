"""Training and weights of the learned precision / solver selector.

The selector (liblsq: lsq_selector_set / lsq_selector_features, inference in
a HIP kernel) maps 16 features of an instance to a factorization precision
{FP8-e4m3, BF16, FP16, FP32, FP64 direct} and a refinement solver {classical
IR, GMRES-IR}.  The features are cheap: the sizes, the FP64 norms of the
inputs, and the diagonal statistics of the triangles of the instance's FP32
generalized factorization, the first rung of the plain ladder, whose factors
the FP32 rungs then reuse.

Labels come from the method itself: every instance of a generated set is
solved once per rung (escalation off) on the batch workers, and the label is
the rung that certifies a backward error <= 1e-14 at the least cost to AUTO,
which is the rung's own time for an FP32 rung and the FP32 factorization plus
the rung's time for any other.

    python -m paper_2406_16499_amd.selector collect --count 50000 --seed 5 --out data.npz
    python -m paper_2406_16499_amd.selector fit --data data.npz
    python -m paper_2406_16499_amd.selector evaluate --count 5000 --seed 6

Weights are stored as text (one value per line, the packed order of
LSQ_SELECTOR_WEIGHTS) in selector_weights.txt next to this file; Handle()
loads them when present.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
WEIGHTS_PATH = os.path.join(HERE, "selector_weights.txt")
NF, NH, NO = 16, 64, 7
N_WEIGHTS = 2 * NF + NH * NF + NH + NH * NH + NH + NO * NH + NO
# precision classes and solver classes of the two heads
PREC_CLASSES = ["fp8", "bf16", "fp16", "fp32", "fp64"]
NP = len(PREC_CLASSES)
SOLVER_CLASSES = ["ir", "gmres"]
# rungs tried when labelling; the features come from the FP32 factorization
RUNGS = [("fp8", "ir"), ("fp8", "gmres"), ("bf16", "ir"), ("bf16", "gmres"), ("fp16", "ir"),
         ("fp16", "gmres"), ("fp32", "ir"), ("fp32", "gmres"), ("fp64", "direct")]
FEATURE_PREC = "fp32"
REUSES_FEATURE_FACTORS = np.array([p == FEATURE_PREC for p, _ in RUNGS])


# ----------------------------------------------------------------- model --
def init_params(rng):
    def he(o, i):
        return (rng.standard_normal((o, i)) * math.sqrt(2.0 / i)).astype(np.float32)
    return {"mean": np.zeros(NF, np.float32), "std": np.ones(NF, np.float32),
            "W1": he(NH, NF), "b1": np.zeros(NH, np.float32),
            "W2": he(NH, NH), "b2": np.zeros(NH, np.float32),
            "W3": he(NO, NH) * 0.1, "b3": np.zeros(NO, np.float32)}


def pack(P) -> np.ndarray:
    w = np.concatenate([P["mean"], P["std"], P["W1"].ravel(), P["b1"], P["W2"].ravel(), P["b2"],
                        P["W3"].ravel(), P["b3"]]).astype(np.float32)
    assert w.size == N_WEIGHTS
    return w


def unpack(w) -> dict:
    w = np.asarray(w, np.float32)
    assert w.size == N_WEIGHTS
    out, o = {}, 0
    for name, shape in (("mean", (NF,)), ("std", (NF,)), ("W1", (NH, NF)), ("b1", (NH,)),
                        ("W2", (NH, NH)), ("b2", (NH,)), ("W3", (NO, NH)), ("b3", (NO,))):
        k = int(np.prod(shape))
        out[name] = w[o:o + k].reshape(shape)
        o += k
    return out


def forward(P, X):
    """Logits (n x 6) in FP32, the same arithmetic as the HIP kernel."""
    Xn = (X - P["mean"]) / P["std"]
    h1 = np.maximum(Xn @ P["W1"].T + P["b1"], 0.0)
    h2 = np.maximum(h1 @ P["W2"].T + P["b2"], 0.0)
    return h2 @ P["W3"].T + P["b3"], (Xn, h1, h2)


def predict(P, X):
    lo, _ = forward(P, np.asarray(X, np.float32))
    return np.argmax(lo[:, :NP], axis=1), np.argmax(lo[:, NP:], axis=1)


def _softmax_ce(z, y):
    z = z - z.max(axis=1, keepdims=True)
    e = np.exp(z)
    pr = e / e.sum(axis=1, keepdims=True)
    loss = -np.log(pr[np.arange(len(y)), y] + 1e-12).mean()
    g = pr.copy()
    g[np.arange(len(y)), y] -= 1.0
    return loss, g / len(y)


def train(X, yp, ys, epochs=400, lr=3e-3, seed=0, wd=1e-4):
    """Full-batch Adam on the sum of the two heads' cross-entropies."""
    X = np.asarray(X, np.float32)
    rng = np.random.default_rng(seed)
    P = init_params(rng)
    P["mean"] = X.mean(axis=0).astype(np.float32)
    P["std"] = (X.std(axis=0) + 1e-3).astype(np.float32)
    keys = ["W1", "b1", "W2", "b2", "W3", "b3"]
    m = {k: np.zeros_like(P[k]) for k in keys}
    v = {k: np.zeros_like(P[k]) for k in keys}
    hist = []
    for it in range(1, epochs + 1):
        lo, (Xn, h1, h2) = forward(P, X)
        l1, g1 = _softmax_ce(lo[:, :NP], yp)
        l2, g2 = _softmax_ce(lo[:, NP:], ys)
        gz = np.concatenate([g1, g2], axis=1).astype(np.float32)
        G = {"W3": gz.T @ h2, "b3": gz.sum(0)}
        gh2 = (gz @ P["W3"]) * (h2 > 0)
        G["W2"], G["b2"] = gh2.T @ h1, gh2.sum(0)
        gh1 = (gh2 @ P["W2"]) * (h1 > 0)
        G["W1"], G["b1"] = gh1.T @ Xn, gh1.sum(0)
        for k in keys:
            g = G[k] + wd * P[k]
            m[k] = 0.9 * m[k] + 0.1 * g
            v[k] = 0.999 * v[k] + 0.001 * g * g
            mh, vh = m[k] / (1 - 0.9 ** it), v[k] / (1 - 0.999 ** it)
            P[k] = (P[k] - lr * mh / (np.sqrt(vh) + 1e-8)).astype(np.float32)
        hist.append(float(l1 + l2))
    return P, hist


def save(P, path=WEIGHTS_PATH, meta=None):
    w = pack(P)
    with open(path, "w") as fh:
        fh.write("# selector weights: MLP 16-64-64-7, packed order mean, std, W1, b1, W2, b2, W3, b3\n")
        if meta:
            fh.write("# " + json.dumps(meta) + "\n")
        for x in w:
            fh.write(f"{x:.9g}\n")


def load(path=WEIGHTS_PATH):
    vals = [float(l) for l in open(path) if l.strip() and not l.startswith("#")]
    return np.asarray(vals, np.float32)


# ----------------------------------------------------- data from the GPU --
def _generate(args):
    """Instances [start, stop) of the batch recipe (runs in a worker process,
    one BLAS thread)."""
    seed, start, stop, kappa_max = args
    from threadpoolctl import threadpool_limits
    from . import workloads as wl
    with threadpool_limits(1):
        return list(wl.batch_instances(seed=seed, count=stop, kappa_max=kappa_max, start=start))


def instance_stream(count, seed, kappa_max, chunk, procs=12, sub=50):
    """Chunks of `chunk` instances, generated by `procs` worker processes while
    the caller works on the previous chunk (at most two chunks in flight)."""
    import multiprocessing as mp
    from collections import deque
    from concurrent.futures import ProcessPoolExecutor
    spans = [(s, min(s + sub, count)) for s in range(0, count, sub)]
    per_chunk = max(1, chunk // sub)
    with ProcessPoolExecutor(max_workers=procs, mp_context=mp.get_context("spawn")) as pool:
        pending = deque()
        nxt = 0

        def fill():
            nonlocal nxt
            while nxt < len(spans) and len(pending) < 2 * per_chunk:
                a, b = spans[nxt]
                pending.append(pool.submit(_generate, (seed, a, b, kappa_max)))
                nxt += 1
        fill()
        while pending:
            out = []
            for _ in range(min(per_chunk, len(pending))):
                out.extend(pending.popleft().result())
            fill()
            yield out


def _device_problem(P):
    from . import lsq
    if P.kind == "lse":
        t = tuple(lsq.colmajor(a) for a in (P.A, P.B, P.b, P.d))
        x = lsq.empty(P.shape[1])
        return lsq.make_problem("lse", t, x), (t, x)
    t = tuple(lsq.colmajor(a) for a in (P.W, P.V, P.d))
    x, y = lsq.empty(P.shape[1]), lsq.empty(P.shape[2])
    return lsq.make_problem("gls", t, x, y), (t, x, y)


def features(h, P):
    desc, keep = _device_problem(P)
    return h.selector_features(desc)[0]


def label_chunk(h, descs, maxit=20, gmres_maxit=60, log=None):
    """(T, OK, TF) for instances already on the device: per rung of RUNGS the
    solve time (ms: conversion + factorization + refinement, event-timed on
    the batch worker that ran it) and whether it certified at that rung, and
    the FP32 factorization time (conversion + factorization of the fp32/ir
    solve)."""
    from . import lsq
    n = len(descs)
    T = np.full((n, len(RUNGS)), np.inf)
    OK = np.zeros((n, len(RUNGS)), bool)
    TF = np.full(n, np.inf)
    h.set_batch_mode("workers")
    for j, (prec, solver) in enumerate(RUNGS):
        opts = lsq.default_opts(prec=prec, solver=solver, escalate=0, maxit=maxit,
                                gmres_maxit=gmres_maxit)
        t0 = time.perf_counter()
        rc, res = h.lsq_solve_batched(descs, opts)
        for i, r in enumerate(res):
            T[i, j] = r.ms_convert + r.ms_factor + r.ms_refine
            OK[i, j] = (r.info == 0 and r.berr_max <= 1e-14 and lsq.PREC_NAME[r.prec_used] == prec
                        and lsq.SOLVER_NAME[r.solver_used] == solver)
            if (prec, solver) == (FEATURE_PREC, "ir"):
                TF[i] = r.ms_convert + r.ms_factor
        if log:
            log(f"  rung {prec}/{solver}: {int(OK[:, j].sum())}/{n} certified, "
                f"{time.perf_counter() - t0:.1f} s")
    h.set_batch_mode("persistent")
    return T, OK, TF


TIMES = {}   # mode -> [seconds, certified] summed over the chunks of the last collect


def time_modes(h, descs, weights, log=None):
    """Wall-clock seconds and certified counts of one pass over descs on the
    batch workers for AUTO (selector weights set), the plain ladder (FP32
    classical IR, then GMRES-IR, then FP64 direct) and FP64 direct."""
    import torch
    from . import lsq
    h.set_batch_mode("workers")
    modes = {"auto": lsq.default_opts(prec="auto", solver="auto", escalate=1),
             "ladder": lsq.default_opts(prec="fp32", solver="ir", escalate=1),
             "fp64": lsq.default_opts(prec="fp64", solver="direct")}
    out = {}
    for name, opts in modes.items():
        h.selector_set(weights if name == "auto" else None)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rc, res = h.lsq_solve_batched(descs, opts)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        ok = sum(1 for r in res if r.info == 0 and r.berr_max <= 1e-14)
        out[name] = (dt, ok)
        if log:
            log(f"  {name}: {dt:.2f} s, {ok}/{len(descs)} certified")
    h.selector_set(None)
    h.set_batch_mode("persistent")
    return out


def collect(h, count, seed, kappa_max=1e12, chunk=2000, out=None, log=None, procs=12, weights=None):
    """Features and labels of `count` instances of the batch recipe.  h is a
    Handle, or a callable returning one: it is then called after the generator
    processes have started, so that they are not started from a process that
    already holds the GPU."""
    import torch
    X, T, OK, TF, META = [], [], [], [], []
    TIMES.clear()
    done = 0
    stream = instance_stream(count, seed, kappa_max, chunk, procs)
    first = next(stream, None)
    if callable(h):
        h = h()

    def chunks():
        if first is not None:
            yield first
            yield from stream
    for probs in chunks():
        t0 = time.perf_counter()
        up = [_device_problem(P) for P in probs]
        descs = [d for d, _ in up]
        torch.cuda.synchronize()
        X.extend(h.selector_features(d)[0] for d in descs)
        if log:
            log(f"chunk at {done}: {len(probs)} instances on the device, features in "
                f"{time.perf_counter() - t0:.1f} s")
        if weights is not None:
            for name, (dt, okc) in time_modes(h, descs, weights, log).items():
                acc = TIMES.setdefault(name, [0.0, 0])
                acc[0] += dt
                acc[1] += okc
        t, ok, tf = label_chunk(h, descs, log=log)
        T.append(t); OK.append(ok); TF.append(tf)
        META.extend([(0 if P.kind == "lse" else 1, *P.shape,
                      getattr(P, "kappa_A", None) or getattr(P, "kappa_W", None) or 0.0,
                      getattr(P, "kappa_B", None) or getattr(P, "kappa_V", None) or 0.0)
                     for P in probs])
        done += len(probs)
        del up, descs
        torch.cuda.empty_cache()
        if out:
            np.savez(out, X=np.array(X, np.float32), T=np.concatenate(T), OK=np.concatenate(OK),
                     TF=np.concatenate(TF), META=np.array(META, float))
        if log:
            log(f"labelled {done}/{count}")
    return (np.array(X, np.float32), np.concatenate(T), np.concatenate(OK), np.concatenate(TF),
            np.array(META, float))


def auto_cost(T, TF):
    """AUTO's cost of starting at each rung: the features come from the FP32
    factorization, which the FP32 rungs keep and every other rung pays on top
    of its own solve."""
    return np.where(REUSES_FEATURE_FACTORS[None, :], T, T + TF[:, None])


def targets(T, OK, TF=None):
    """Cheapest certified rung per instance (AUTO's cost when TF is given, the
    rung's own time otherwise) -> (precision class, solver class); FP64 direct
    counts as the solver class IR.  Instances that no rung certified are
    dropped."""
    C = auto_cost(T, TF) if TF is not None else T
    keep, yp, ys = [], [], []
    for i in range(len(C)):
        if not OK[i].any():
            continue
        j = int(np.argmin(np.where(OK[i], C[i], np.inf)))
        prec, solver = RUNGS[j]
        keep.append(i)
        yp.append(PREC_CLASSES.index(prec))
        ys.append(SOLVER_CLASSES.index(solver if solver in SOLVER_CLASSES else "ir"))
    return np.array(keep, int), np.array(yp, int), np.array(ys, int)


def rung_of(pc, sc):
    """Index in RUNGS of the rung the selector's classes start at."""
    prec = PREC_CLASSES[pc]
    return RUNGS.index((prec, "direct" if prec == "fp64" else SOLVER_CLASSES[sc]))


def fit(data, out=WEIGHTS_PATH, epochs=600, seed=0, meta=None):
    d = np.load(data)
    X, T, OK, TF = d["X"], d["T"], d["OK"], d["TF"]
    keep, yp, ys = targets(T, OK, TF)
    P, hist = train(X[keep], yp, ys, epochs=epochs, seed=seed)
    pp, ps = predict(P, X[keep])
    acc = float(np.mean((pp == yp) & (ps == ys)))
    counts = {f"{PREC_CLASSES[p]}/{SOLVER_CLASSES[s]}": int(np.sum((yp == p) & (ys == s)))
              for p in range(NP) for s in range(2)}
    save(P, out, dict(meta or {}, trained_on=int(len(keep)), train_joint_accuracy=acc,
                      final_loss=hist[-1], label_counts=counts))
    return {"trained_on": int(len(keep)), "joint_accuracy": acc, "label_counts": counts}


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("action", choices=["collect", "fit", "evaluate"])
    ap.add_argument("--count", type=int, default=2000)
    ap.add_argument("--seed", type=int, default=5)
    ap.add_argument("--kappa-max", type=float, default=1e12)
    ap.add_argument("--chunk", type=int, default=2000)
    ap.add_argument("--data", default=None, help="features/labels (.npz)")
    ap.add_argument("--out", default=None)
    a = ap.parse_args(argv)
    log = lambda s: print(s, flush=True)  # noqa: E731
    if a.action == "fit":
        print(json.dumps(fit(a.data, a.out or WEIGHTS_PATH,
                             meta={"data": os.path.basename(a.data)})))
        return
    from . import lsq
    h = lambda: lsq.Handle(load_selector=False)  # noqa: E731
    if a.action == "collect":
        collect(h, a.count, a.seed, a.kappa_max, a.chunk, a.out, log)
        return
    # evaluate: the selector's first pick on a fresh stream, against the
    # labels of the same instances
    wts = load(a.out or WEIGHTS_PATH)
    P = unpack(wts)
    X, T, OK, TF, _ = collect(h, a.count, a.seed, a.kappa_max, a.chunk, a.data, log, weights=wts)
    keep, yp, ys = targets(T, OK, TF)
    pp, ps = predict(P, X[keep])
    C = auto_cost(T, TF)
    picks = [rung_of(pp[j], ps[j]) for j in range(len(keep))]
    first_ok = float(np.mean([OK[i][picks[j]] for j, i in enumerate(keep)]))
    print(json.dumps({"instances": a.count, "wall_s": {k: round(v[0], 3) for k, v in TIMES.items()},
                      "certified": {k: v[1] for k, v in TIMES.items()},
                      "evaluated": int(len(keep)), "first_pick_certifies": first_ok,
                      "joint_accuracy": float(np.mean((pp == yp) & (ps == ys))),
                      "regret_ms_when_certified": float(np.mean(
                          [C[i][picks[j]] - C[i][rung_of(yp[j], ys[j])]
                           for j, i in enumerate(keep) if OK[i][picks[j]]]))}))


if __name__ == "__main__":
    main()
