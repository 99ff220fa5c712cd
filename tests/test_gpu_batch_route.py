"""The launch shape of the persistent batch: the diagonal-ratio route that
sends an instance from the FP32 rung straight to FP64, the longest instances
that the FP64 rung takes from the start, both set directly and through the
size-bucket table, and the FP64 share of the compute units.
Every setting must certify every instance against the oracle; only the rung
that solves an instance may change."""
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


@pytest.fixture(scope="module")
def batch():
    probs = list(wl.batch_instances(seed=83, count=24, kappa_max=1e6, m_range=(64, 300)))
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
    return probs, keep, descs


def _solve_check(h, batch):
    probs, keep, descs = batch
    rc, res = h.lsq_solve_batched(descs, lsq.default_opts(prec="fp32", escalate=1))
    assert rc == 0, (rc, h.last_error())
    for P, (t, x, y), r in zip(probs, keep, res):
        assert r.info == 0 and r.berr_max <= 1e-14, r.as_dict()
        if P.kind == "lse":
            xo, ro, vo = direct.lse_solve(P.A, P.B, P.b, P.d)
            assert _fwd(x.cpu().numpy(), xo) <= 10 * direct.lse_cond_x(P.A, P.B, xo, ro, vo) * U64
        else:
            xo, yo, zo = direct.gls_solve(P.W, P.V, P.d)
            cx, cy = direct.gls_cond_xy(P.W, P.V, xo, yo, zo)
            assert _fwd(x.cpu().numpy(), xo) <= 10 * cx * U64
            assert _fwd(y.cpu().numpy(), yo) <= 10 * cy * U64
    return [(r.as_dict()["prec_used"], r.attempts) for r in res]


def test_route_off_keeps_every_instance_on_fp32(h, batch):
    note("route off, 24 instances kappa<=1e6")
    h.dbg_batch_route(0.0)
    rungs = _solve_check(h, batch)
    assert all(r == ("fp32", 1) for r in rungs), rungs


def test_route_at_one_sends_every_instance_to_fp64(h, batch):
    # the ratio of the largest to the smallest diagonal entry of a triangular
    # factor exceeds 1 for every generated instance
    note("route 1.0, 24 instances")
    h.dbg_batch_route(1.0)
    try:
        rungs = _solve_check(h, batch)
    finally:
        h.dbg_batch_route(3e5)
    assert all(r == ("fp64", 2) for r in rungs), rungs


def test_tuning_table_overrides_the_route_for_its_bucket(h, batch):
    note("table: bucket <= 300 routes at 1.0; bucket <= 200 (not covering) off")
    h.dbg_batch_route(0.0)
    try:
        h.batch_tuning([(200, 0.0, 0.25), (300, 1.0, 0.125)])
        assert all(r == ("fp64", 2) for r in _solve_check(h, batch))
        h.batch_tuning([(1024, 0.0, 0.3125)])
        assert all(r == ("fp32", 1) for r in _solve_check(h, batch))
        h.batch_tuning([(100, 1.0, 0.25)])          # no entry covers the batch
        assert all(r == ("fp32", 1) for r in _solve_check(h, batch))
    finally:
        h.batch_tuning([])
        h.dbg_batch_route(3e5)


def _work(P):
    # the longest-first order of the batched entry points (factorization flops)
    if P.kind == "lse":
        m, n, p = P.shape
        return 2 * m * n * n + 4 * m * n * p + 2 * n * p * p
    n, m, p = P.shape
    return 2 * n * m * m + 4 * n * m * p + 2 * p * n * n


@pytest.mark.parametrize("per_wg,count", [(0.25, 6), (8.0, 21)])
def test_pre_sends_the_longest_instances_to_fp64(h, batch, per_wg, count):
    # share 1/4 of 256 compute units: 64 FP64 work-groups, capped at the 24
    # instances, so per_wg x 24 instances (rounded) go to FP64 at once, at
    # most 21 (7/8 of the batch: the shortest 3 always try FP32)
    note(f"pre {per_wg}: {count} of 24 instances FP64 from the start")
    probs = batch[0]
    longest = set(sorted(range(len(probs)), key=lambda i: -_work(probs[i]))[:count])
    h.dbg_batch_route(0.0)
    h.dbg_batch_pre(per_wg)
    try:
        rungs = _solve_check(h, batch)
    finally:
        h.dbg_batch_pre(0.0)
        h.dbg_batch_route(3e5)
    for i, r in enumerate(rungs):
        assert r == (("fp64", 1) if i in longest else ("fp32", 1)), (i, r)


def test_tuning_table_sets_pre_for_its_bucket(h, batch):
    note("table: bucket <= 300 with pre 0.25")
    probs = batch[0]
    longest = set(sorted(range(len(probs)), key=lambda i: -_work(probs[i]))[:6])
    try:
        h.batch_tuning([(300, 0.0, 0.25, 0.25)])
        rungs = _solve_check(h, batch)
    finally:
        h.batch_tuning([])
    for i, r in enumerate(rungs):
        assert r == (("fp64", 1) if i in longest else ("fp32", 1)), (i, r)


def test_pre_with_escalations(h):
    # FP64-first instances and FP32 failures share the FP64 rung's queues
    note("pre 0.25 with escalations, 20 instances kappa<=1e12")
    probs = list(wl.batch_instances(seed=85, count=20, kappa_max=1e12, m_range=(64, 300)))
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
    longest = set(sorted(range(len(probs)), key=lambda i: -_work(probs[i]))[:5])
    h.dbg_batch_pre(0.25)
    try:
        rungs = _solve_check(h, (probs, keep, descs))
    finally:
        h.dbg_batch_pre(0.0)
    assert any(r == ("fp64", 2) for r in rungs), rungs
    for i, r in enumerate(rungs):
        if i in longest:
            assert r == ("fp64", 1), (i, r)
        else:
            assert r in (("fp32", 1), ("fp64", 2)), (i, r)


def _make(probs):
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
    return probs, keep, descs


def test_escalation_regime_picks_the_entry(h, batch):
    # two entries for one bucket: one for any regime (6 of the 24 longest
    # instances FP64 first), one while at most 2% escalated (none first)
    note("regime: entry for any regime, then the low-escalation entry, then back")
    probs = batch[0]
    longest = set(sorted(range(len(probs)), key=lambda i: -_work(probs[i]))[:6])
    ill = _make(list(wl.batch_instances(seed=85, count=20, kappa_max=1e12, m_range=(64, 300))))
    h.dbg_batch_route(0.0)
    try:
        h.batch_tuning([(300, 0.0, 0.25, 0.25, 1.0), (300, 0.0, 0.25, 0.0, 0.02)])
        assert h.dbg_batch_regime() == 1.0
        for i, r in enumerate(_solve_check(h, batch)):
            assert r == (("fp64", 1) if i in longest else ("fp32", 1)), (i, r)
        assert h.dbg_batch_regime() == 0.0
        assert all(r == ("fp32", 1) for r in _solve_check(h, batch))
        rungs = _solve_check(h, ill)
        assert all(r in (("fp32", 1), ("fp64", 2)) for r in rungs), rungs
        failed = sum(r == ("fp64", 2) for r in rungs)
        assert failed >= 1 and h.dbg_batch_regime() == failed / len(rungs)
        for i, r in enumerate(_solve_check(h, batch)):
            assert r == (("fp64", 1) if i in longest else ("fp32", 1)), (i, r)
        h.batch_tuning([(300, 0.0, 0.25, 0.25, 1.0), (300, 0.0, 0.25, 0.0, 0.02)])
        assert h.dbg_batch_regime() == 1.0      # a new table starts from the top regime
    finally:
        h.batch_tuning([])
        h.dbg_batch_route(3e5)


@pytest.mark.parametrize("share", [0.0625, 0.5])
def test_fp64_share_keeps_results_certified(h, share):
    note(f"fp64 share {share}, 20 instances kappa<=1e12")
    probs = list(wl.batch_instances(seed=84, count=20, kappa_max=1e12, m_range=(64, 300)))
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
    h.dbg_batch_split(share)
    try:
        rungs = _solve_check(h, (probs, keep, descs))
    finally:
        h.dbg_batch_split(0.25)
    assert any(r[0] == "fp64" for r in rungs)
