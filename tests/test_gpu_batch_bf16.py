"""The persistent batch with a BF16 factorization (trailing updates and the
first factorization's Q^T applied with BF16 MFMA inputs, FP32 accumulation):
well-conditioned pairs certify on the BF16 rung alone, in more refinement
steps than on the FP32 rung (the lower precision is in effect); with
escalation every instance certifies, on the BF16 rung or in FP64."""
import sys

import numpy as np
import pytest

from oracle import direct
from paper_2406_16499_amd import lsq
from paper_2406_16499_amd import workloads as wl

pytestmark = pytest.mark.gpu
U64 = 2.0 ** -53


def note(msg):
    sys.stdout.write(f"\n[case] {msg}\n")
    sys.stdout.flush()


@pytest.fixture(scope="module")
def h():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    hd = lsq.Handle(load_selector=False, load_tuning=False)
    hd.set_batch_mode("persistent")
    yield hd
    hd.close()


def _fwd(a, ref):
    return np.max(np.abs(a - ref)) / np.max(np.abs(ref))


def _descriptors(probs):
    keep, descs = [], []
    for P in probs:
        if P.kind == "lse":
            t = tuple(lsq.colmajor(a) for a in (P.A, P.B, P.b, P.d))
            x, y = lsq.empty(P.shape[1]), None
            descs.append(lsq.make_problem("lse", t, x))
        else:
            t = tuple(lsq.colmajor(a) for a in (P.W, P.V, P.d))
            x, y = lsq.empty(P.shape[1]), lsq.empty(P.shape[2])
            descs.append(lsq.make_problem("gls", t, x, y))
        keep.append((t, x, y))
    return keep, descs


def _check(P, x, y, r):
    assert r.info == 0 and r.berr_max <= 1e-14, r.as_dict()
    if P.kind == "lse":
        xo, ro, vo = direct.lse_solve(P.A, P.B, P.b, P.d)
        assert _fwd(x.cpu().numpy(), xo) <= 10 * direct.lse_cond_x(P.A, P.B, xo, ro, vo) * U64
    else:
        xo, yo, zo = direct.gls_solve(P.W, P.V, P.d)
        cx, cy = direct.gls_cond_xy(P.W, P.V, xo, yo, zo)
        assert _fwd(x.cpu().numpy(), xo) <= 10 * cx * U64
        assert _fwd(y.cpu().numpy(), yo) <= 10 * cy * U64


def _well_conditioned():
    rng = np.random.default_rng(94)
    probs = []
    for (m, n, p) in [(96, 32, 4), (128, 48, 8), (160, 40, 12), (200, 64, 16), (70, 33, 5), (250, 17, 3)]:
        probs.append(wl.lse_conditioned(rng, m, n, p, 1.0, 1.0))
    for (n, m, p) in [(96, 24, 80), (130, 40, 100), (64, 9, 60), (200, 50, 180)]:
        probs.append(wl.gls_conditioned(rng, n, m, p, 1.0, 1.0))
    return probs


def test_bf16_rung_alone_certifies_well_conditioned_pairs(h):
    note("bf16 persistent, escalate 0, 10 pairs kappa 1")
    probs = _well_conditioned()
    keep, descs = _descriptors(probs)
    rc, res = h.lsq_solve_batched(descs, lsq.default_opts(prec="bf16", solver="ir", escalate=0))
    assert rc == 0, h.last_error()
    for P, (t, x, y), r in zip(probs, keep, res):
        _check(P, x, y, r)
        d = r.as_dict()
        assert (d["prec_used"], d["solver_used"], d["attempts"]) == ("bf16", "ir", 1), d
    steps16 = np.array([r.ir_steps for r in res])
    rc, res32 = h.lsq_solve_batched(descs, lsq.default_opts(prec="fp32", solver="ir", escalate=0))
    assert rc == 0
    steps32 = np.array([r.ir_steps for r in res32])
    assert all(r.as_dict()["prec_used"] == "fp32" for r in res32)
    note(f"steps bf16 {steps16.tolist()} fp32 {steps32.tolist()}")
    assert steps16.mean() > steps32.mean() + 1, (steps16, steps32)


def test_bf16_first_with_escalation_certifies_every_instance(h):
    note("bf16 persistent with escalation, 24 instances kappa<=1e4 and the 10 kappa-1 pairs")
    probs = list(wl.batch_instances(seed=95, count=24, kappa_max=1e4, m_range=(64, 300))) + _well_conditioned()
    keep, descs = _descriptors(probs)
    rc, res = h.lsq_solve_batched(descs, lsq.default_opts(prec="bf16", solver="ir", escalate=1))
    assert rc == 0, h.last_error()
    for P, (t, x, y), r in zip(probs, keep, res):
        _check(P, x, y, r)
        d = r.as_dict()
        assert (d["prec_used"], d["attempts"]) in (("bf16", 1), ("fp64", 2)), d
    assert any(r.as_dict()["prec_used"] == "fp64" for r in res)
