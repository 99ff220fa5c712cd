"""The selector on the GPU: features, the HIP MLP kernel against the numpy
forward pass, and AUTO solves through the C-ABI."""
import sys

import numpy as np
import pytest

from oracle import direct
from paper_2406_16499_amd import lsq
from paper_2406_16499_amd import selector as sel
from paper_2406_16499_amd import workloads as wl

pytestmark = pytest.mark.gpu


def note(msg):
    sys.stdout.write(f"\n[case] {msg}\n")
    sys.stdout.flush()


@pytest.fixture(scope="module")
def h():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    hd = lsq.Handle(load_selector=False)
    yield hd
    hd.close()


def _weights(seed=3):
    rng = np.random.default_rng(seed)
    P = sel.init_params(rng)
    P["mean"] = (rng.standard_normal(16) * 0.5).astype(np.float32)
    P["std"] = (rng.random(16) + 0.5).astype(np.float32)
    P["W3"] = (rng.standard_normal((sel.NO, 64)) * 0.3).astype(np.float32)
    P["b3"] = (rng.standard_normal(sel.NO) * 0.1).astype(np.float32)
    return P


@pytest.mark.parametrize("seed", [50, 51, 52, 53])
def test_features_and_mlp_kernel(h, seed):
    P = next(iter(wl.batch_instances(seed=seed, count=1, kappa_max=1e6, m_range=(64, 300))))
    note(f"selector features {wl.describe(P)}")
    desc, keep = sel._device_problem(P)
    W = _weights(seed)
    h.selector_set(sel.pack(W))
    f, lo, cls = h.selector_features(desc, with_logits=True)
    if P.kind == "lse":
        m, n, p = P.shape
        A, B, vecs = P.A, P.B, (np.linalg.norm(P.b), np.linalg.norm(P.d))
        # the triangle of the RQ of B is (up to the index reversal J) the R of
        # the QR of J B^T J, whose diagonal magnitudes are those of QR(B^T J)
        R = np.linalg.qr(B.T[:, ::-1], mode="r")
        t = 0
    else:
        n, m, p = P.shape
        A, B, vecs = P.W, P.V, (np.linalg.norm(P.d), 0.0)
        R = np.linalg.qr(P.W, mode="r")
        t = 1
    assert f[0] == t
    assert np.allclose(f[1:4], np.log2(np.array([m, n, p]) + 1.0), rtol=1e-6)
    assert f[4] == pytest.approx(np.log10(np.linalg.norm(A)), abs=1e-5)
    assert f[5] == pytest.approx(np.log10(np.linalg.norm(B)), abs=1e-5)
    if vecs[0] > 0:
        assert f[6] == pytest.approx(np.log10(vecs[0]), abs=1e-5)
    d = np.abs(np.diag(R))
    assert f[8] == pytest.approx(np.log10(d.max() / d.min()), abs=0.1)   # BF16 factors
    ref, _ = sel.forward(W, f[None, :])
    assert np.allclose(lo, ref[0], rtol=1e-4, atol=1e-4)
    assert cls == [int(np.argmax(ref[0, :sel.NP])), int(np.argmax(ref[0, sel.NP:]))]


def test_selector_set_rejects_bad_weights(h):
    note("selector_set errors")
    w = sel.pack(_weights())
    assert h.lib.lsq_selector_set(h.h, None, 0) == 0
    import ctypes
    short = np.ascontiguousarray(w[:100])
    assert h.lib.lsq_selector_set(h.h, short.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), 100) == -3
    bad = w.copy()
    bad[16] = 0.0                                         # a zero feature scale
    assert h.lib.lsq_selector_set(h.h, bad.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), bad.size) == -2


@pytest.mark.parametrize("cls_bias", [0, 1, 2, 3, 4])
def test_auto_solves_certify_whatever_the_pick(h, cls_bias):
    # weights whose output forces one precision class: the ladder must still
    # certify every instance (the selector's pick is only a starting rung)
    note(f"auto solve forced class {cls_bias}")
    W = _weights()
    W["W3"][:] = 0.0
    W["b3"][:] = 0.0
    W["b3"][cls_bias] = 5.0
    W["b3"][sel.NP + (cls_bias % 2)] = 5.0
    h.selector_set(sel.pack(W))
    probs = list(wl.batch_instances(seed=60 + cls_bias, count=6, kappa_max=1e7, m_range=(64, 256)))
    keep, descs = [], []
    for P in probs:
        d, k = sel._device_problem(P)
        descs.append(d)
        keep.append(k)
    rc, res = h.lsq_solve_batched(descs, lsq.default_opts(prec="auto", solver="auto"))
    assert rc == 0, h.last_error()
    for P, k, r in zip(probs, keep, res):
        assert r.info == 0 and r.berr_max <= 1e-14
        x = k[1].cpu().numpy()
        if P.kind == "lse":
            assert direct.lse_err1(P.B, P.d, x) <= 1e-13
        else:
            assert direct.gls_err1(P.W, P.V, P.d, x, k[2].cpu().numpy()) <= 1e-13
    first = {lsq.PREC_NAME[r.prec_used] for r in res if r.attempts == 1}
    want = {0: "fp8", 1: "bf16", 2: "fp16", 3: "fp32", 4: "fp64"}[cls_bias]
    assert first <= {want}
    h.selector_set(None)
