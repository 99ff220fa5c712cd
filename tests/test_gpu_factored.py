"""Factor once, solve many: lse_factor / gls_factor then *_solve_factored on
several right-hand sides, against the oracle; switching between classical IR
and GMRES-IR on the same factors; error paths of the entry points."""
import sys
import time

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
    hd.close()


def D(a):
    return lsq.colmajor(a)


def H(t):
    return t.detach().cpu().numpy()


def _fwd(a, ref):
    s = np.max(np.abs(ref)) if ref.size else 0.0
    d = np.max(np.abs(a - ref)) if ref.size else 0.0
    return d / s if s > 0 else d


def _check_lse(A, B, b, d, x, r, v, res):
    assert res.berr_max <= 1e-14
    be = direct.lse_berr(A, B, b, d, x, r, v)
    assert be[3] <= 1.01e-14
    xo, ro, vo = direct.lse_solve(A, B, b, d)
    cond = direct.lse_cond_x(A, B, xo, ro, vo)
    assert _fwd(x, xo) <= 10 * cond * U64


def _check_gls(W, V, d, x, y, z, res):
    assert res.berr_max <= 1e-14
    be = direct.gls_berr(W, V, d, x, y, z)
    assert be[3] <= 1.01e-14
    xo, yo, zo = direct.gls_solve(W, V, d)
    cx, cy = direct.gls_cond_xy(W, V, xo, yo, zo)
    assert _fwd(x, xo) <= 10 * cx * U64
    assert _fwd(y, yo) <= 10 * cy * U64


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_lse_factor_once_many_rhs(h, prec):
    # several panels and a ragged tail; three right-hand sides on one factorization
    m, n, p = 300, 200, 40
    note(f"lse factored {prec} m={m} n={n} p={p}")
    rng = np.random.default_rng(101)
    # u_f kappa(A) kappa(B) ~ 0.1 for BF16, inside the GMRES preconditioner's bound
    P = wl.lse_conditioned(rng, m, n, p, 1e3 if prec == "fp32" else 10.0)
    A, B = D(P.A), D(P.B)
    F = h.lse_factor(A, B, prec)
    try:
        for j, solver in enumerate(["ir", "ir", "gmres", "ir"]):
            b, d = rng.standard_normal(m), rng.standard_normal(p)
            x, r, v = lsq.empty(n), lsq.empty(m), lsq.empty(p)
            rc, res = F.solve(D(b), D(d), x, r, v, opts=lsq.default_opts(solver=solver))
            dd = res.as_dict()
            assert rc == 0, (j, solver, rc, h.last_error(), dd)
            assert dd["prec_used"] == prec and dd["solver_used"] == solver and dd["attempts"] == 1
            assert res.ms_factor == 0.0
            _check_lse(P.A, P.B, b, d, H(x), H(r), H(v), res)
    finally:
        F.close()


def test_gls_factor_once_many_rhs(h):
    n, m, p = 260, 120, 300
    note(f"gls factored fp32 n={n} m={m} p={p}")
    rng = np.random.default_rng(102)
    G = wl.gls_conditioned(rng, n, m, p, 1e3)
    F = h.gls_factor(D(G.W), D(G.V), "fp32")
    try:
        for j, solver in enumerate(["ir", "gmres", "ir"]):
            d = rng.standard_normal(n)
            x, y, z = lsq.empty(m), lsq.empty(p), lsq.empty(n)
            rc, res = F.solve(D(d), x, y, z, opts=lsq.default_opts(solver=solver))
            dd = res.as_dict()
            assert rc == 0, (j, solver, rc, h.last_error(), dd)
            assert dd["solver_used"] == solver and res.ms_factor == 0.0
            _check_gls(G.W, G.V, d, H(x), H(y), H(z), res)
    finally:
        F.close()


def test_factored_fp64_runs_the_direct_solve(h):
    m, n, p = 150, 90, 30
    note("lse factored fp64")
    rng = np.random.default_rng(103)
    P = wl.lse_gaussian(rng, m, n, p)
    F = h.lse_factor(D(P.A), D(P.B), "fp64")
    try:
        x, r, v = lsq.empty(n), lsq.empty(m), lsq.empty(p)
        rc, res = F.solve(D(P.b), D(P.d), x, r, v)
        assert rc == 0 and res.as_dict()["solver_used"] == "direct"
        _check_lse(P.A, P.B, P.b, P.d, H(x), H(r), H(v), res)
    finally:
        F.close()


def test_factored_matches_full_solve(h):
    # the same precision and solver through lse_solve: both land on the FP64 solution
    m, n, p = 400, 256, 64
    note("lse factored vs lse_solve")
    P = wl.config2(seed=5, m=m, n=n, p=p, kappa=1e3)
    A, B = D(P.A), D(P.B)
    x1, x2 = lsq.empty(n), lsq.empty(n)
    rc1, _ = h.lse_solve(A, B, D(P.b), D(P.d), x1, None, None,
                         lsq.default_opts(prec="fp32", solver="ir", escalate=0))
    F = h.lse_factor(A, B, "fp32")
    try:
        rc2, _ = F.solve(D(P.b), D(P.d), x2)
    finally:
        F.close()
    assert rc1 == 0 and rc2 == 0
    xo, _, _ = direct.lse_solve(P.A, P.B, P.b, P.d)
    assert _fwd(H(x1), xo) <= 1e-10 and _fwd(H(x2), xo) <= 1e-10


def test_factored_solve_skips_the_factorization(h):
    # on a factorization-dominated shape a factored solve costs a fraction of a full one
    import torch
    m, n, p = 4096, 1024, 128
    note("lse factored timing 4096x1024x128")
    P = wl.config2(seed=6, m=m, n=n, p=p, kappa=1e3)
    A, B, b, d = D(P.A), D(P.B), D(P.b), D(P.d)
    x = lsq.empty(n)
    o = lsq.default_opts(prec="fp32", solver="ir", escalate=0)
    h.lse_solve(A, B, b, d, x, None, None, o)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rc, _ = h.lse_solve(A, B, b, d, x, None, None, o)
    t_full = time.perf_counter() - t0
    F = h.lse_factor(A, B, "fp32")
    try:
        F.solve(b, d, x, opts=o)
        t0 = time.perf_counter()
        rc2, res = F.solve(b, d, x, opts=o)
        t_fac = time.perf_counter() - t0
    finally:
        F.close()
    assert rc == 0 and rc2 == 0
    assert t_fac < 0.8 * t_full, (t_fac, t_full)


def test_factored_error_paths(h):
    note("factored error paths")
    lib = h.lib
    P = wl.lse_gaussian(np.random.default_rng(104), 40, 30, 10)
    A, B = D(P.A), D(P.B)
    import ctypes
    f = ctypes.c_void_p()
    assert lib.lse_factor(h.h, 40, 30, 10, lsq._ptr(A), 40, lsq._ptr(B), 10, lsq.PREC["auto"],
                          ctypes.byref(f)) == -9
    assert lib.lse_factor(h.h, 40, 30, 10, lsq._ptr(A), 40, lsq._ptr(B), 10, lsq.PREC["fp32"],
                          None) == -10
    assert lib.lse_factor(h.h, 40, 50, 5, lsq._ptr(A), 40, lsq._ptr(B), 10, lsq.PREC["fp32"],
                          ctypes.byref(f)) == -3
    F = h.lse_factor(A, B, "fp32")
    try:
        x = lsq.empty(30)
        rc, _ = F.solve(D(P.b), D(P.d), x, opts=lsq.default_opts(solver="direct"))
        assert rc == -8                                   # DIRECT needs FP64 factors
        res = lsq.Result()
        assert lib.lse_solve_factored(h.h, F.f, None, lsq._ptr(D(P.d)), lsq._ptr(x), None, None,
                                      None, ctypes.byref(res)) == -3
        assert lib.gls_solve_factored(h.h, F.f, lsq._ptr(D(P.d)), lsq._ptr(x), lsq._ptr(x), None,
                                      None, ctypes.byref(res)) == -2   # LSE factors
        h2 = lsq.Handle(load_selector=False)
        try:
            assert lib.lse_solve_factored(h2.h, F.f, lsq._ptr(D(P.b)), lsq._ptr(D(P.d)), lsq._ptr(x),
                                          None, None, None, ctypes.byref(res)) == -2
        finally:
            h2.close()
    finally:
        F.close()
    assert lib.lsq_factors_destroy(None) == 0
