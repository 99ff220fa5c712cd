"""Deterministic mode (lsq_dbg_deterministic): the same input gives bitwise
identical output, run after run, for the single solves (classical IR and
GMRES-IR) and the batched workers; the default mode agrees with it to the
oracle's bound."""
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
    hd = lsq.Handle(load_selector=False)
    yield hd
    hd.lib.lsq_dbg_deterministic(hd.h, 0)
    hd.close()


def D(a):
    return lsq.colmajor(a)


def H(t):
    return t.detach().cpu().numpy()


def _lse(h, P, opts):
    m, n, p = P.shape
    x, r, v = lsq.empty(n), lsq.empty(m), lsq.empty(p)
    rc, res = h.lse_solve(D(P.A), D(P.B), D(P.b), D(P.d), x, r, v, opts)
    assert rc == 0 and res.berr_max <= 1e-14, res.as_dict()
    return H(x), H(r), H(v), tuple(res.berr)


def _gls(h, G, opts):
    n, m, p = G.shape
    x, y, z = lsq.empty(m), lsq.empty(p), lsq.empty(n)
    rc, res = h.gls_solve(D(G.W), D(G.V), D(G.d), x, y, z, opts)
    assert rc == 0 and res.berr_max <= 1e-14, res.as_dict()
    return H(x), H(y), H(z), tuple(res.berr)


def _same(a, b):
    return all(np.array_equal(u, v) for u, v in zip(a[:3], b[:3])) and a[3] == b[3]


def test_lse_classical_ir_bitwise(h):
    note("determinism lse fp32 ir 700x300x40 kappa 1e5")
    P = wl.lse_conditioned(np.random.default_rng(801), 700, 300, 40, 1e5)
    opts = lsq.default_opts(prec="fp32", solver="ir", escalate=0)
    h.lib.lsq_dbg_deterministic(h.h, 1)
    runs = [_lse(h, P, opts) for _ in range(3)]
    h.lib.lsq_dbg_deterministic(h.h, 0)
    assert _same(runs[0], runs[1]) and _same(runs[0], runs[2])
    default = _lse(h, P, opts)
    xo, ro, vo = direct.lse_solve(P.A, P.B, P.b, P.d)
    cond = direct.lse_cond_x(P.A, P.B, xo, ro, vo)
    for x in (runs[0][0], default[0]):
        assert np.max(np.abs(x - xo)) <= 10 * cond * U64 * np.max(np.abs(xo))


def test_gls_gmres_ir_bitwise(h):
    note("determinism gls fp32 gmres 500x120x450 kappa 1e6")
    G = wl.gls_conditioned(np.random.default_rng(802), 500, 120, 450, 1e6)
    opts = lsq.default_opts(prec="fp32", solver="gmres", escalate=0)
    h.lib.lsq_dbg_deterministic(h.h, 1)
    runs = [_gls(h, G, opts) for _ in range(2)]
    h.lib.lsq_dbg_deterministic(h.h, 0)
    assert _same(runs[0], runs[1])
    xo, yo, zo = direct.gls_solve(G.W, G.V, G.d)
    cx, cy = direct.gls_cond_xy(G.W, G.V, xo, yo, zo)
    assert np.max(np.abs(runs[0][0] - xo)) <= 10 * cx * U64 * np.max(np.abs(xo))
    assert np.max(np.abs(runs[0][1] - yo)) <= 10 * cy * U64 * np.max(np.abs(yo))


def test_batched_workers_bitwise(h):
    note("determinism batched workers 24 instances")
    probs = list(wl.batch_instances(seed=803, count=24, kappa_max=1e6, m_range=(64, 400)))
    from paper_2406_16499_amd import selector as sel
    ups = [sel._device_problem(P) for P in probs]
    descs = [d for d, _ in ups]
    h.lib.lsq_dbg_deterministic(h.h, 1)
    h.set_batch_mode("workers")
    outs = []
    for _ in range(2):
        rc, res = h.lsq_solve_batched(descs, lsq.default_opts(prec="fp32", solver="ir"))
        assert rc == 0 and all(r.info == 0 and r.berr_max <= 1e-14 for r in res)
        outs.append([H(k[1]).copy() for _, k in ups])
    h.set_batch_mode("persistent")
    h.lib.lsq_dbg_deterministic(h.h, 0)
    for a, b in zip(*outs):
        assert np.array_equal(a, b)
