"""CPU checks of the selector's model code (training and the packed layout);
the HIP inference kernel is compared with `forward` in test_gpu_selector."""
import numpy as np

from paper_2406_16499_amd import selector as sel


def test_pack_unpack_roundtrip_and_size():
    P = sel.init_params(np.random.default_rng(0))
    w = sel.pack(P)
    assert w.size == sel.N_WEIGHTS == 5735
    Q = sel.unpack(w)
    for k in P:
        assert np.array_equal(P[k], Q[k])


def test_header_constant_matches():
    import re
    import os
    txt = open(os.path.join(os.path.dirname(sel.HERE), "include", "lsq.h")).read()
    assert int(re.search(r"#define LSQ_SELECTOR_WEIGHTS (\d+)", txt).group(1)) == sel.N_WEIGHTS
    assert int(re.search(r"#define LSQ_SELECTOR_FEATURES (\d+)", txt).group(1)) == sel.NF


def test_forward_matches_plain_loops():
    rng = np.random.default_rng(1)
    P = sel.init_params(rng)
    P["mean"] = rng.standard_normal(16).astype(np.float32)
    P["std"] = (rng.random(16) + 0.5).astype(np.float32)
    x = rng.standard_normal(16).astype(np.float32)
    lo, _ = sel.forward(P, x[None, :])
    xn = [(x[i] - P["mean"][i]) / P["std"][i] for i in range(16)]
    h1 = [max(0.0, sum(P["W1"][j][i] * xn[i] for i in range(16)) + P["b1"][j]) for j in range(64)]
    h2 = [max(0.0, sum(P["W2"][j][i] * h1[i] for i in range(64)) + P["b2"][j]) for j in range(64)]
    ref = [sum(P["W3"][c][i] * h2[i] for i in range(64)) + P["b3"][c] for c in range(sel.NO)]
    assert np.allclose(lo[0], ref, rtol=1e-4, atol=1e-5)


def test_training_separates_a_synthetic_rule():
    # precision class from feature 10 (a condition estimate), solver from feature 0
    rng = np.random.default_rng(2)
    X = rng.standard_normal((1500, 16)).astype(np.float32)
    X[:, 10] = rng.uniform(0, 12, 1500)
    X[:, 0] = rng.integers(0, 2, 1500)
    yp = np.digitize(X[:, 10], [2.4, 4.8, 7.2, 9.6])
    ys = X[:, 0].astype(int)
    P, hist = sel.train(X, yp, ys, epochs=600)
    pp, ps = sel.predict(P, X)
    assert hist[-1] < hist[0]
    assert np.mean(pp == yp) > 0.9 and np.mean(ps == ys) > 0.98


def test_targets_pick_cheapest_certified_rung_for_auto():
    # RUNGS: fp8 ir/gmres, bf16 ir/gmres, fp16 ir/gmres, fp32 ir/gmres, fp64 direct
    assert [r for r in sel.RUNGS if r[0] == sel.FEATURE_PREC] == [("fp32", "ir"), ("fp32", "gmres")]
    T = np.array([[1.0, 2, 3, 4, 5, 6, 7, 8, 9],
                  [1.0, 2, 3, 4, 5, 6, 7, 8, 0.5],
                  [1.0] * 9,
                  [9.0, 9, 9, 9, 9, 9, 6, 9, 2]])
    OK = np.array([[False, False, True, False, True, True, True, True, True], [True] * 9, [False] * 9,
                   [True] * 9])
    TF = np.array([10.0, 0.1, 1.0, 5.0])
    # own times: row 0 -> bf16/ir (3), row 1 -> fp64 (0.5), row 3 -> fp64 (2)
    keep, yp, ys = sel.targets(T, OK)
    assert list(keep) == [0, 1, 3]
    assert [(sel.PREC_CLASSES[p], sel.SOLVER_CLASSES[s]) for p, s in zip(yp, ys)] == \
        [("bf16", "ir"), ("fp64", "ir"), ("fp64", "ir")]
    # AUTO pays the FP32 factorization (TF) on top of every non-FP32 rung:
    # row 0: bf16/ir 13 vs fp32/ir 7 -> fp32/ir; row 1: fp8/ir 1.1 vs fp64 0.6 -> fp64;
    # row 3: fp64 7 vs fp32/ir 6 -> fp32/ir
    C = sel.auto_cost(T, TF)
    assert C[0, 2] == 13.0 and C[0, 6] == 7.0 and C[3, 8] == 7.0 and C[3, 6] == 6.0
    keep, yp, ys = sel.targets(T, OK, TF)
    assert list(keep) == [0, 1, 3]
    assert [(sel.PREC_CLASSES[p], sel.SOLVER_CLASSES[s]) for p, s in zip(yp, ys)] == \
        [("fp32", "ir"), ("fp64", "ir"), ("fp32", "ir")]
    assert [sel.rung_of(p, s) for p, s in zip(yp, ys)] == [6, 8, 6]


def test_instance_stream_matches_the_generator():
    from paper_2406_16499_amd import workloads as wl
    chunks = list(sel.instance_stream(7, seed=11, kappa_max=1e12, chunk=4, procs=2, sub=2))
    assert [len(c) for c in chunks] == [4, 3]
    ref = list(wl.batch_instances(seed=11, count=7, kappa_max=1e12))
    got = [P for c in chunks for P in c]
    for P, Q in zip(got, ref):
        assert P.kind == Q.kind and P.shape == Q.shape
        a, b = (P.A, Q.A) if P.kind == "lse" else (P.W, Q.W)
        # the same instance up to the rounding of multi- vs single-threaded BLAS
        assert np.allclose(a, b, rtol=1e-12, atol=1e-14 * np.max(np.abs(b)))
