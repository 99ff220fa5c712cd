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


def test_targets_pick_fastest_certified_rung():
    T = np.array([[1.0, 2.0, 3.0, 4.0, 5.0, 6.0, 7.0], [1.0, 2.0, 3.0, 4.0, 0.5, 6.0, 7.0],
                  [1, 1, 1, 1, 1, 1, 1.0], [5, 5, 5, 5, 5, 5, 0.1]])
    OK = np.array([[False, True, True, False, True, True, True], [True] * 7, [False] * 7,
                   [True] * 7])
    keep, yp, ys = sel.targets(T, OK)
    assert list(keep) == [0, 1, 3]
    assert (sel.PREC_CLASSES[yp[0]], sel.SOLVER_CLASSES[ys[0]]) == ("bf16", "gmres")
    assert (sel.PREC_CLASSES[yp[1]], sel.SOLVER_CLASSES[ys[1]]) == ("fp32", "ir")
    assert sel.PREC_CLASSES[yp[2]] == "fp64"
