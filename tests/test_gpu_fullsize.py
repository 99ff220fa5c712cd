"""Parity at the full sizes the benchmark times, against the CPU oracle.

- the large LSE: A 4096 x 2048 with kappa(A) = 1e4, B 256 x 2048 (seed 2),
  FP32 factorization with classical IR and the BF16 ladder;
- the large GLS: W 4096 x 1024, V 4096 x 4096 with kappa(V) = 1e6 (seed 3),
  FP16 and BF16 factorizations with GMRES-IR and the ladder;
- the 4096 x 1024 x 128 LSE factored once and solved on stored factors.

Each solution is compared element by element with the oracle's: the
backward error is recomputed by the oracle (<= 1e-14) and the forward error
of x (GLS: x and y) is bounded by 10 kappa 2^-53, with kappa the Skeel
condition number of the block (estimated by the block 1-norm estimator, as
the augmented systems have 6400 and 9216 unknowns).  The launch
configuration is the one bench.py times (default options, one handle)."""
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
    hd.close()


def D(a):
    return lsq.colmajor(a)


def H(t):
    return t.detach().cpu().numpy()


def _fwd(a, ref):
    s = np.max(np.abs(ref)) if ref.size else 0.0
    d = np.max(np.abs(a - ref)) if ref.size else 0.0
    return d / s if s > 0 else d


@pytest.fixture(scope="module")
def lse_large():
    # oracle solution and the Skeel condition numbers of its r, v and x blocks
    P = wl.config2()
    m, n, p = P.shape
    xo, ro, vo = direct.lse_solve(P.A, P.B, P.b, P.d)
    F = direct.lse_augmented(P.A, P.B)
    u = np.concatenate([ro, -vo, xo])
    conds = [direct.skeel_cond_block_est(F, u, sl)
             for sl in (slice(0, m), slice(m, m + p), slice(m + p, m + p + n))]
    return P, (xo, ro, vo), conds


@pytest.fixture(scope="module")
def gls_large():
    # oracle solution and the Skeel condition numbers of its y, z and x blocks
    G = wl.config3()
    n, m, p = G.shape
    xo, yo, zo = direct.gls_solve(G.W, G.V, G.d)
    F = direct.gls_augmented(G.W, G.V)
    u = np.concatenate([yo, -zo, xo])
    conds = [direct.skeel_cond_block_est(F, u, sl)
             for sl in (slice(0, p), slice(p, p + n), slice(p + n, p + n + m))]
    return G, (xo, yo, zo), conds


@pytest.mark.parametrize("prec,solver,escalate", [("fp32", "ir", 1), ("bf16", "ir", 1)])
def test_lse_4096x2048x256(h, lse_large, prec, solver, escalate):
    P, (xo, ro, vo), (cr, cv, cond) = lse_large
    note(f"lse 4096x2048x256 {prec} {solver} escalate={escalate} (cond r, v, x ~ {cr:.3g}, {cv:.3g}, {cond:.3g})")
    m, n, p = P.shape
    x, r, v = lsq.empty(n), lsq.empty(m), lsq.empty(p)
    rc, res = h.lse_solve(D(P.A), D(P.B), D(P.b), D(P.d), x, r, v,
                          lsq.default_opts(prec=prec, solver=solver, escalate=escalate))
    assert rc == 0, (rc, h.last_error(), res.as_dict())
    sys.stdout.write(f"[result] {res.as_dict()}\n")
    x, r, v = H(x), H(r), H(v)
    be = direct.lse_berr(P.A, P.B, P.b, P.d, x, r, v)
    assert res.berr_max <= 1e-14 and be[3] <= 1e-14, (res.berr_max, be)
    assert _fwd(x, xo) <= 10 * cond * U64, (_fwd(x, xo), cond)
    assert _fwd(r, ro) <= 10 * cr * U64, (_fwd(r, ro), cr)
    assert _fwd(v, vo) <= 10 * cv * U64, (_fwd(v, vo), cv)
    if prec == "fp32":
        assert res.as_dict()["prec_used"] == "fp32" and res.attempts == 1


@pytest.mark.parametrize("prec", ["fp16", "bf16"])
def test_gls_4096x1024x4096_gmres(h, gls_large, prec):
    G, (xo, yo, zo), (cy, cz, cx) = gls_large
    note(f"gls 4096x1024x4096 {prec} gmres ladder (cond y, z, x ~ {cy:.3g}, {cz:.3g}, {cx:.3g})")
    n, m, p = G.shape
    x, y, z = lsq.empty(m), lsq.empty(p), lsq.empty(n)
    rc, res = h.gls_solve(D(G.W), D(G.V), D(G.d), x, y, z,
                          lsq.default_opts(prec=prec, solver="gmres", escalate=1))
    assert rc == 0, (rc, h.last_error(), res.as_dict())
    sys.stdout.write(f"[result] {res.as_dict()}\n")
    x, y, z = H(x), H(y), H(z)
    be = direct.gls_berr(G.W, G.V, G.d, x, y, z)
    assert res.berr_max <= 1e-14 and be[3] <= 1e-14, (res.berr_max, be)
    assert _fwd(x, xo) <= 10 * cx * U64, (_fwd(x, xo), cx)
    assert _fwd(y, yo) <= 10 * cy * U64, (_fwd(y, yo), cy)
    assert _fwd(z, zo) <= 10 * cz * U64, (_fwd(z, zo), cz)
    assert res.as_dict()["solver_used"] == "gmres"


def test_lse_factored_4096x1024x128(h):
    P = wl.config2(seed=6, m=4096, n=1024, p=128, kappa=1e3)
    m, n, p = P.shape
    note("lse factored 4096x1024x128 fp32: three right-hand sides")
    F = h.lse_factor(D(P.A), D(P.B), "fp32")
    try:
        g = np.random.default_rng(61)
        for j in range(3):
            b, d = g.standard_normal(m), g.standard_normal(p)
            x, r, v = lsq.empty(n), lsq.empty(m), lsq.empty(p)
            rc, res = F.solve(D(b), D(d), x, r, v, opts=lsq.default_opts(prec="fp32", solver="ir", escalate=0))
            assert rc == 0, (j, rc, res.as_dict())
            xo, ro, vo = direct.lse_solve(P.A, P.B, b, d)
            cond = direct.lse_cond_x_est(P.A, P.B, xo, ro, vo)
            be = direct.lse_berr(P.A, P.B, b, d, H(x), H(r), H(v))
            assert be[3] <= 1e-14
            assert _fwd(H(x), xo) <= 10 * cond * U64, (j, _fwd(H(x), xo), cond)
    finally:
        F.close()
