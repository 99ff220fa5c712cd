"""Persistent batched execution (one work-group per instance): every instance
certified against the oracle, the in-kernel FP32 -> FP64 escalation, the edge
shapes of both problems, and the hand-over of ineligible or failing instances
to the batch workers."""
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
    # the launch-shape table is a performance setting: these tests pin the
    # escalation mechanism itself (FP32 first for every instance)
    hd = lsq.Handle(load_tuning=False)
    hd.set_batch_mode("persistent")
    yield hd
    hd.close()


def _fwd(a, ref):
    s = np.max(np.abs(ref)) if ref.size else 0.0
    d = np.max(np.abs(a - ref)) if ref.size else 0.0
    return d / s if s > 0 else d


def _descriptors(probs):
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


def _check(P, x, y, res, tol=1e-14):
    assert res.info == 0 and res.berr_max <= tol, res.as_dict()
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


def _run(h, probs, **opts):
    keep, descs = _descriptors(probs)
    rc, res = h.lsq_solve_batched(descs, lsq.default_opts(**opts))
    out = [(x.cpu().numpy(), None if y is None else y.cpu().numpy()) for (t, x, y) in keep]
    return rc, res, out


def test_persistent_mixed_batch_certifies_every_instance(h):
    note("persistent 40 mixed instances kappa<=1e6")
    probs = list(wl.batch_instances(seed=70, count=40, kappa_max=1e6, m_range=(64, 500)))
    rc, res, out = _run(h, probs, prec="fp32")
    assert rc == 0, (rc, h.last_error())
    for P, (x, y), r in zip(probs, out, res):
        _check(P, x, y, r)
        d = r.as_dict()
        assert d["prec_used"] == "fp32" and d["solver_used"] == "ir" and d["attempts"] == 1


def test_persistent_escalates_to_fp64_inside_the_batch(h):
    # kappa up to 1e12 is beyond FP32 refinement for part of the batch: those
    # instances are factored again in FP64 by the second persistent launch
    note("persistent 24 instances kappa<=1e12 escalation")
    probs = list(wl.batch_instances(seed=71, count=24, kappa_max=1e12, m_range=(64, 300)))
    rc, res, out = _run(h, probs, prec="fp32", escalate=1)
    assert rc == 0, (rc, h.last_error())
    precs = [r.as_dict()["prec_used"] for r in res]
    assert "fp64" in precs and "fp32" in precs
    for P, (x, y), r in zip(probs, out, res):
        _check(P, x, y, r)
        d = r.as_dict()
        if d["prec_used"] == "fp64":
            assert d["solver_used"] == "direct" and d["attempts"] == 2


def test_persistent_fp64_only(h):
    note("persistent fp64 12 instances")
    probs = list(wl.batch_instances(seed=72, count=12, kappa_max=1e10, m_range=(64, 300)))
    rc, res, out = _run(h, probs, prec="fp64", solver="direct")
    assert rc == 0, (rc, h.last_error())
    for P, (x, y), r in zip(probs, out, res):
        _check(P, x, y, r)
        d = r.as_dict()
        assert d["prec_used"] == "fp64" and d["attempts"] == 1 and d["ir_steps"] <= 2


def _lse(rng, m, n, p, kappa=1e2):
    return wl.lse_conditioned(rng, m, n, p, kappa)


def _gls(rng, n, m, p, kappa=1e2):
    return wl.gls_conditioned(rng, n, m, p, kappa)


def test_persistent_edge_shapes(h):
    # n = p (no T11), m < n, one-row B, GLS with n = m, p < n, the largest
    # eligible dimensions and a ragged 65-row case
    note("persistent edge shapes")
    rng = np.random.default_rng(73)
    probs = [
        _lse(rng, 40, 12, 12),        # k = n - p = 0
        _lse(rng, 20, 30, 15),        # m < n
        _lse(rng, 1, 2, 1),           # smallest: m = 1
        _lse(rng, 65, 33, 1),         # one constraint, ragged rows
        _lse(rng, 1024, 96, 24),      # largest eligible m
        _gls(rng, 30, 30, 10),        # n = m: k = 0
        _gls(rng, 50, 20, 35),        # p < n
        _gls(rng, 2, 1, 1),           # smallest
        _gls(rng, 130, 7, 1024),      # largest eligible p
        _gls(rng, 64, 64, 64),        # square blocks
    ]
    rc, res, out = _run(h, probs, prec="fp32")
    assert rc == 0, (rc, h.last_error())
    for P, (x, y), r in zip(probs, out, res):
        _check(P, x, y, r)


def test_persistent_hands_ineligible_instances_to_the_workers(h):
    # an instance with m > 1024 runs on the batch workers; the rest persistent
    note("persistent + worker hand-over")
    rng = np.random.default_rng(74)
    probs = [_lse(rng, 1100, 64, 8), _gls(rng, 80, 20, 60), _lse(rng, 300, 100, 10)]
    rc, res, out = _run(h, probs, prec="fp32")
    assert rc == 0, (rc, h.last_error())
    for P, (x, y), r in zip(probs, out, res):
        _check(P, x, y, r)


def test_persistent_without_escalation_reports_the_failure(h):
    # kappa 1e10 with FP32 only: the instance goes to the worker ladder, which
    # (escalate = 0) reports info 3; the well-conditioned one is certified
    note("persistent escalate=0")
    rng = np.random.default_rng(75)
    probs = [_lse(rng, 200, 60, 10, kappa=1e10), _lse(rng, 200, 60, 10, kappa=1e2)]
    rc, res, out = _run(h, probs, prec="fp32", escalate=0)
    assert rc == 1
    assert res[0].info == 3 and res[1].info == 0
    _check(probs[1], out[1][0], None, res[1])


def test_persistent_matches_worker_mode(h):
    note("persistent vs workers")
    probs = list(wl.batch_instances(seed=76, count=10, kappa_max=1e5, m_range=(64, 400)))
    rc1, res1, out1 = _run(h, probs, prec="fp32")
    h.set_batch_mode("workers")
    try:
        rc2, res2, out2 = _run(h, probs, prec="fp32")
    finally:
        h.set_batch_mode("persistent")
    assert rc1 == 0 and rc2 == 0
    for P, a, b, r1, r2 in zip(probs, out1, out2, res1, res2):
        _check(P, a[0], a[1], r1)
        _check(P, b[0], b[1], r2)
        xo = direct.lse_solve(P.A, P.B, P.b, P.d)[0] if P.kind == "lse" else \
            direct.gls_solve(P.W, P.V, P.d)[0]
        assert _fwd(a[0], b[0]) <= 2.5 * max(_fwd(a[0], xo), _fwd(b[0], xo)) + 1e-15


def test_persistent_workspace_reuse_smaller_second_batch(h):
    note("persistent two calls, the second smaller")
    big = list(wl.batch_instances(seed=77, count=12, kappa_max=1e4, m_range=(300, 700)))
    small = list(wl.batch_instances(seed=78, count=5, kappa_max=1e4, m_range=(64, 100)))
    for probs in (big, small):
        rc, res, out = _run(h, probs, prec="fp32")
        assert rc == 0, (rc, h.last_error())
        for P, (x, y), r in zip(probs, out, res):
            _check(P, x, y, r)


def test_persistent_concurrent_fp64_rung_matches_sequential(h):
    # the FP64 rung beside the FP32 launch solves the same instances as a
    # second launch would, with the same kernels: the same rungs, and both
    # results certified (the residual's column sums are LDS atomics, so two
    # runs agree to rounding, not bit for bit)
    note("persistent concurrent vs sequential escalation")
    probs = list(wl.batch_instances(seed=79, count=30, kappa_max=1e12, m_range=(64, 400)))
    rc1, res1, out1 = _run(h, probs, prec="fp32", escalate=1)
    h.set_batch_mode("sequential")
    try:
        rc2, res2, out2 = _run(h, probs, prec="fp32", escalate=1)
    finally:
        h.set_batch_mode("persistent")
    assert rc1 == 0 and rc2 == 0
    assert "fp64" in [r.as_dict()["prec_used"] for r in res1]
    for P, a, b, r1, r2 in zip(probs, out1, out2, res1, res2):
        d1, d2 = r1.as_dict(), r2.as_dict()
        assert (d1["prec_used"], d1["attempts"]) == (d2["prec_used"], d2["attempts"])
        _check(P, a[0], a[1], r1)
        _check(P, b[0], b[1], r2)


def test_persistent_fp64_rung_after_the_fp32_launch(h):
    # FP64 work-groups that may not wait leave at once; the work-groups that
    # follow the FP32 launch solve the queued instances and every instance
    # certifies
    note("persistent escalation, early consumers leave at once")
    probs = list(wl.batch_instances(seed=80, count=20, kappa_max=1e12, m_range=(64, 300)))
    h.dbg_batch_wait(0.0)
    try:
        rc, res, out = _run(h, probs, prec="fp32", escalate=1)
    finally:
        h.dbg_batch_wait(50.0)
    assert rc == 0, (rc, h.last_error())
    precs = [r.as_dict()["prec_used"] for r in res]
    assert "fp64" in precs
    for P, (x, y), r in zip(probs, out, res):
        _check(P, x, y, r)
        d = r.as_dict()
        if d["prec_used"] == "fp64":
            assert d["solver_used"] == "direct" and d["attempts"] == 2
