"""Batched execution: many LSE/GLS instances of uneven size through
lsq_solve_batched, each checked against the oracle."""
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
    # without the launch-shape table: these tests pin the FP32-first rungs
    hd = lsq.Handle(load_tuning=False)
    yield hd
    hd.close()


def _fwd(a, ref):
    s = np.max(np.abs(ref)) if ref.size else 0.0
    d = np.max(np.abs(a - ref)) if ref.size else 0.0
    return d / s if s > 0 else d


def _descriptors(probs):
    """Device tensors and descriptors for a list of instances."""
    keep, descs = [], []
    for P in probs:
        if P.kind == "lse":
            m, n, p = P.shape
            t = tuple(lsq.colmajor(a) for a in (P.A, P.B, P.b, P.d))
            x = lsq.empty(n)
            descs.append(lsq.make_problem("lse", t, x))
            keep.append((t, x, None))
        else:
            n, m, p = P.shape
            t = tuple(lsq.colmajor(a) for a in (P.W, P.V, P.d))
            x, y = lsq.empty(m), lsq.empty(p)
            descs.append(lsq.make_problem("gls", t, x, y))
            keep.append((t, x, y))
    return keep, descs


def _check(P, x, y, res):
    assert res.info == 0 and res.berr_max <= 1e-14, res.as_dict()
    if P.kind == "lse":
        xo, ro, vo = direct.lse_solve(P.A, P.B, P.b, P.d)
        assert direct.lse_err1(P.B, P.d, x) <= 1e-13
        cond = direct.lse_cond_x(P.A, P.B, xo, ro, vo)
        assert _fwd(x, xo) <= 10 * cond * U64
    else:
        xo, yo, zo = direct.gls_solve(P.W, P.V, P.d)
        assert direct.gls_err1(P.W, P.V, P.d, x, y) <= 1e-13
        cx, cy = direct.gls_cond_xy(P.W, P.V, xo, yo, zo)
        assert _fwd(x, xo) <= 10 * cx * U64
        assert _fwd(y, yo) <= 10 * cy * U64


@pytest.mark.parametrize("mode,workers", [("workers", 1), ("workers", 4), ("workers", 8),
                                          ("persistent", 8)])
def test_batched_mixed_fp32(h, mode, workers):
    note(f"batched 20 mixed instances fp32 mode={mode} workers={workers}")
    probs = list(wl.batch_instances(seed=40, count=20, kappa_max=1e4, m_range=(64, 300)))
    keep, descs = _descriptors(probs)
    assert h.lib.lsq_set_batch_workers(h.h, workers) == 0
    h.set_batch_mode(mode)
    try:
        rc, res = h.lsq_solve_batched(descs, lsq.default_opts(prec="fp32"))
    finally:
        h.set_batch_mode("persistent")
    assert rc == 0, (rc, h.last_error())
    for P, (t, x, y), r in zip(probs, keep, res):
        _check(P, x.cpu().numpy(), None if y is None else y.cpu().numpy(), r)
        assert r.as_dict()["prec_used"] == "fp32"


def test_batched_bf16_with_ladder(h):
    # kappa up to 1e8: BF16 classical IR cannot reach every instance; the
    # ladder on the batch workers (GMRES-IR on the same factors, then higher
    # precisions) must (the persistent batch goes from BF16 straight to FP64)
    note("batched 16 instances bf16 kappa<=1e8, workers")
    probs = list(wl.batch_instances(seed=41, count=16, kappa_max=1e8, m_range=(64, 400)))
    keep, descs = _descriptors(probs)
    assert h.lib.lsq_set_batch_workers(h.h, 8) == 0
    h.set_batch_mode("workers")
    try:
        rc, res = h.lsq_solve_batched(descs, lsq.default_opts(prec="bf16", solver="ir", escalate=1))
    finally:
        h.set_batch_mode("persistent")
    assert rc == 0, (rc, h.last_error())
    for P, (t, x, y), r in zip(probs, keep, res):
        _check(P, x.cpu().numpy(), None if y is None else y.cpu().numpy(), r)
    assert max(r.attempts for r in res) > 1


def test_batched_matches_single_instance_calls(h):
    note("batched vs single calls")
    probs = list(wl.batch_instances(seed=42, count=6, kappa_max=1e3, m_range=(64, 200)))
    keep, descs = _descriptors(probs)
    rc, res = h.lsq_solve_batched(descs, lsq.default_opts(prec="fp32"))
    assert rc == 0
    for P, (t, x, y), r in zip(probs, keep, res):
        if P.kind == "lse":
            x1 = lsq.empty(P.shape[1])
            rc1, r1 = h.lse_solve(*t, x1, None, None, lsq.default_opts(prec="fp32"))
            assert rc1 == 0
            _check(P, x1.cpu().numpy(), None, r1)
            assert r1.prec_used == r.prec_used and r1.solver_used == r.solver_used
        else:
            x1, y1 = lsq.empty(P.shape[1]), lsq.empty(P.shape[2])
            rc1, r1 = h.gls_solve(*t, x1, y1, None, lsq.default_opts(prec="fp32"))
            assert rc1 == 0
            _check(P, x1.cpu().numpy(), y1.cpu().numpy(), r1)
            assert r1.prec_used == r.prec_used and r1.solver_used == r.solver_used


def test_batched_prebuilt_array_and_raw_results(h):
    # the descriptors marshalled once and the results as the C array: the same
    # rungs and certified results as the list form, on repeated calls
    note("batched prebuilt descriptor array, raw results")
    probs = list(wl.batch_instances(seed=43, count=12, kappa_max=1e6, m_range=(64, 300)))
    keep, descs = _descriptors(probs)
    arr = lsq.problem_array(descs)
    assert len(arr) == len(descs)
    opts = lsq.default_opts(prec="fp32", escalate=1)
    rc, ref = h.lsq_solve_batched(descs, opts)
    assert rc == 0 and isinstance(ref, list)
    for _ in range(2):
        rc, res = h.lsq_solve_batched(arr, opts, raw=True)
        assert rc == 0 and len(res) == len(probs) and not isinstance(res, list)
        for P, (t, x, y), r, r0 in zip(probs, keep, res, ref):
            _check(P, x.cpu().numpy(), None if y is None else y.cpu().numpy(), r)
            assert (r.prec_used, r.solver_used, r.attempts) == (r0.prec_used, r0.solver_used, r0.attempts)


def test_batched_rejects_invalid_descriptor(h):
    note("batched invalid descriptor")
    probs = list(wl.batch_instances(seed=43, count=2, kappa_max=1e2, m_range=(64, 100)))
    keep, descs = _descriptors(probs)
    descs[1].lda = 0
    rc, _ = h.lsq_solve_batched(descs, lsq.default_opts(prec="fp32"))
    assert rc == -3
    assert h.lib.lsq_set_batch_workers(h.h, 0) == -2
    # typed wrappers check the type of every descriptor
    kinds = [P.kind for P in probs]
    if "gls" in kinds:
        rc, _ = h.lsq_solve_batched(descs, lsq.default_opts(prec="fp32"), which="lse")
        assert rc == -3
