"""The allocation-free factored LSE solve (lse_solve_factored_noalloc) against
the allocating one (lse_solve_factored) and the oracle: two calls in a row,
the second on a smaller problem; its error paths; the factors' memory stays
the same size."""
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
    hd.lib.lsq_dbg_noalloc_cap(0)
    hd.close()


def D(a):
    return lsq.colmajor(a)


def H(t):
    return t.detach().cpu().numpy()


def _rel(a, ref):
    s = np.max(np.abs(ref))
    return np.max(np.abs(a - ref)) / s if s > 0 else np.max(np.abs(a))


def _solve_pair(F, b, d, n, m, p, opts):
    """(x, r, v, rc, res) of the allocating and of the allocation-free solve."""
    out = []
    for fn in (F.solve, F.solve_noalloc):
        x, r, v = lsq.empty(n), lsq.empty(m), lsq.empty(p)
        rc, res = fn(D(b), D(d), x, r, v, opts=opts)
        out.append((H(x), H(r), H(v), rc, res))
    return out


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_noalloc_two_calls_match_factored(h, prec):
    rng = np.random.default_rng(404)
    # first call on the larger problem (several 64-column panels, ragged tails),
    # the second on a smaller one: the scratch keeps the first call's contents
    shapes = [(700, 300, 40), (200, 100, 20)]
    probs = [wl.lse_conditioned(rng, m, n, p, 1e3) for (m, n, p) in shapes]
    facs = []
    try:
        for P in probs:
            F = h.lse_factor(D(P.A), D(P.B), prec)
            facs.append(F)
            # prepares the factors for classical refinement (allocates)
            m, n = P.A.shape
            p = P.B.shape[0]
            x, r, v = lsq.empty(n), lsq.empty(m), lsq.empty(p)
            rc, _ = F.solve(D(P.b), D(P.d), x, r, v, opts=lsq.default_opts(solver="ir"))
            assert rc == 0, h.last_error()
        for P, F in zip(probs, facs):
            m, n = P.A.shape
            p = P.B.shape[0]
            note(f"noalloc {prec} m={m} n={n} p={p}")
            used0 = F.bytes()
            b, d = rng.standard_normal(m), rng.standard_normal(p)
            (xf, rf, vf, rcf, resf), (xa, ra, va, rca, resa) = _solve_pair(
                F, b, d, n, m, p, lsq.default_opts(solver="ir"))
            assert rcf == 0, h.last_error()
            assert rca == 0, h.last_error()
            assert resa.info == 0 and resa.berr_max <= 1e-14
            assert F.bytes() == used0                    # nothing allocated in the factors
            be = direct.lse_berr(P.A, P.B, b, d, xa, ra, va)
            assert be[3] <= 1.01e-14
            xo, ro, vo = direct.lse_solve(P.A, P.B, b, d)
            cond = direct.lse_cond_x(P.A, P.B, xo, ro, vo)
            tol = 10 * cond * U64
            assert _rel(xa, xo) <= tol
            assert _rel(xa, xf) <= tol                   # against the allocating entry point
            assert resa.ir_steps == resf.ir_steps
            assert resa.prec_used == resf.prec_used and resa.solver_used == resf.solver_used
    finally:
        for F in facs:
            F.close()


def test_noalloc_error_paths(h):
    rng = np.random.default_rng(405)
    m, n, p = 120, 80, 10
    P = wl.lse_conditioned(rng, m, n, p, 1e2)
    F = h.lse_factor(D(P.A), D(P.B), "fp32")
    try:
        x, r, v = lsq.empty(n), lsq.empty(m), lsq.empty(p)
        note("noalloc unprepared factors")
        rc, _ = F.solve_noalloc(D(P.b), D(P.d), x, r, v)
        assert rc == -2 and "prepared" in h.last_error()
        rc, _ = F.solve(D(P.b), D(P.d), x, r, v, opts=lsq.default_opts(solver="ir"))
        assert rc == 0
        note("noalloc gmres rejected")
        rc, _ = F.solve_noalloc(D(P.b), D(P.d), x, r, v, opts=lsq.default_opts(solver="gmres"))
        assert rc == -8
        note("noalloc workspace cap")
        need, cap = F.noalloc_bytes()
        assert 0 < need <= cap == 64 << 20
        assert h.lib.lsq_dbg_noalloc_cap(need - 256) == 0
        rc, _ = F.solve_noalloc(D(P.b), D(P.d), x, r, v)
        assert rc == -2 and "scratch" in h.last_error()
        assert h.lib.lsq_dbg_noalloc_cap(need) == 0
        rc, res = F.solve_noalloc(D(P.b), D(P.d), x, r, v)
        assert rc == 0 and res.berr_max <= 1e-14, h.last_error()
        assert h.lib.lsq_dbg_noalloc_cap((64 << 20) + 1) == -1
        assert h.lib.lsq_dbg_noalloc_cap(0) == 0
        note("noalloc non-finite rhs")
        bad = P.b.copy()
        bad[3] = np.nan
        rc, res = F.solve_noalloc(D(bad), D(P.d), x, r, v)
        assert rc == 5 and res.info == 5
    finally:
        h.lib.lsq_dbg_noalloc_cap(0)
        F.close()
