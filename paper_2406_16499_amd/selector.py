"""Training and weights of the learned precision / solver selector.

The selector (liblsq: lsq_selector_set / lsq_selector_features, inference in
a HIP kernel) maps 16 features of an instance to a factorization precision
{FP8-e4m3, BF16, FP16, FP32, FP64 direct} and a refinement solver {classical
IR, GMRES-IR}.  Its labels come from the method itself: every instance of a
generated training set is solved once per rung with escalation off, and the
label is the fastest rung that certified a backward error <= 1e-14.

    python -m paper_2406_16499_amd.selector train --count 3000 --seed 5
    python -m paper_2406_16499_amd.selector evaluate --count 1000 --seed 6

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
# rungs tried when labelling (FP8 has no factorization of its own yet: it runs as BF16)
RUNGS = [("bf16", "ir"), ("bf16", "gmres"), ("fp16", "ir"), ("fp16", "gmres"),
         ("fp32", "ir"), ("fp32", "gmres"), ("fp64", "direct")]


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


def label(h, P, maxit=20, gmres_maxit=150):
    """(times, ok) of every rung of RUNGS on one instance, escalation off."""
    import torch
    from . import lsq
    desc, keep = _device_problem(P)
    times, ok = [], []
    for prec, solver in RUNGS:
        opts = lsq.default_opts(prec=prec, solver=solver, escalate=0, maxit=maxit,
                                gmres_maxit=gmres_maxit)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rc, res = h.lsq_solve_batched([desc], opts)
        dt = time.perf_counter() - t0
        r = res[0]
        good = rc == 0 and r.info == 0 and r.berr_max <= 1e-14 and \
            lsq.PREC_NAME[r.prec_used] == prec and lsq.SOLVER_NAME[r.solver_used] == solver
        times.append(dt)
        ok.append(bool(good))
    return np.array(times), np.array(ok)


def make_dataset(h, count, seed, kappa_max=1e12, log=None):
    from . import workloads as wl
    X, T, OK = [], [], []
    for i, P in enumerate(wl.batch_instances(seed=seed, count=count, kappa_max=kappa_max)):
        X.append(features(h, P))
        t, ok = label(h, P)
        T.append(t)
        OK.append(ok)
        if log and (i + 1) % 100 == 0:
            log(f"labelled {i + 1}/{count}")
    return np.array(X), np.array(T), np.array(OK)


def targets(T, OK):
    """Fastest certified rung per instance -> (precision class, solver class);
    FP64 direct counts as the solver class IR.  Instances that no rung
    certified are dropped."""
    keep, yp, ys = [], [], []
    for i in range(len(T)):
        if not OK[i].any():
            continue
        j = int(np.argmin(np.where(OK[i], T[i], np.inf)))
        prec, solver = RUNGS[j]
        keep.append(i)
        yp.append(PREC_CLASSES.index(prec))
        ys.append(SOLVER_CLASSES.index(solver if solver in SOLVER_CLASSES else "ir"))
    return np.array(keep, int), np.array(yp, int), np.array(ys, int)


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("action", choices=["train", "evaluate"])
    ap.add_argument("--count", type=int, default=2000)
    ap.add_argument("--seed", type=int, default=5)
    ap.add_argument("--kappa-max", type=float, default=1e12)
    ap.add_argument("--out", default=WEIGHTS_PATH)
    ap.add_argument("--dump", default=None, help="save features/labels (.npz) here")
    a = ap.parse_args(argv)
    sys.path.insert(0, os.path.dirname(HERE))
    from . import lsq
    h = lsq.Handle(load_selector=False)
    log = lambda s: print(s, flush=True)  # noqa: E731
    if a.action == "train":
        X, T, OK = make_dataset(h, a.count, a.seed, a.kappa_max, log)
        if a.dump:
            np.savez(a.dump, X=X, T=T, OK=OK)
        keep, yp, ys = targets(T, OK)
        P, hist = train(X[keep], yp, ys)
        pp, ps = predict(P, X[keep])
        acc = float(np.mean((pp == yp) & (ps == ys)))
        save(P, a.out, {"count": a.count, "seed": a.seed, "kappa_max": a.kappa_max,
                        "train_joint_accuracy": acc, "final_loss": hist[-1]})
        print(json.dumps({"trained_on": int(len(keep)), "joint_accuracy": acc,
                          "label_counts": {f"{PREC_CLASSES[p]}/{SOLVER_CLASSES[s]}": int(np.sum((yp == p) & (ys == s)))
                                           for p in range(NP) for s in range(2)}}))
    else:
        P = unpack(load(a.out))
        X, T, OK = make_dataset(h, a.count, a.seed, a.kappa_max, log)
        keep, yp, ys = targets(T, OK)
        pp, ps = predict(P, X[keep])
        def rung_of(c, sv):
            prec = PREC_CLASSES[max(1, c)]
            return RUNGS.index((prec, "direct" if prec == "fp64" else SOLVER_CLASSES[sv]))
        first_ok = float(np.mean([OK[i][rung_of(pp[j], ps[j])] for j, i in enumerate(keep)]))
        print(json.dumps({"evaluated": int(len(keep)), "first_pick_certifies": first_ok,
                          "joint_accuracy": float(np.mean((pp == yp) & (ps == ys)))}))


if __name__ == "__main__":
    main()
