"""Complex LSE / GLS (zlse_solve, zgls_solve) through the C-ABI against the
complex oracle, which solves over C with Hermitian transposes and no real
embedding: backward error of the complex problem recomputed by the oracle,
forward error within 10 cond 2^-53, edge shapes and the argument checks."""
import sys

import numpy as np
import pytest

from oracle import complex_lsq as zc
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


def C(a):
    return lsq.colmajor_c(a)


def H(t):
    return t.detach().cpu().numpy()


def _rel(a, ref):
    s = np.max(np.abs(ref)) if ref.size else 0.0
    d = np.max(np.abs(a - ref)) if ref.size else 0.0
    return d / s if s > 0 else d


def crandn(rng, *shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def conditioned_c(rng, r, c, kappa):
    """U diag(s) V^H with Haar-unitary U, V (QR of complex Gaussians, phase
    fixed) and s log-spaced from 1 to 1/kappa."""
    k = min(r, c)
    U, Ru = np.linalg.qr(crandn(rng, r, k))
    U = U * (np.diag(Ru) / np.abs(np.diag(Ru)))
    V, Rv = np.linalg.qr(crandn(rng, c, k))
    V = V * (np.diag(Rv) / np.abs(np.diag(Rv)))
    s = kappa ** (-np.arange(k) / max(k - 1, 1))
    return (U * s) @ V.conj().T


@pytest.mark.parametrize("prec,solver", [("fp32", "ir"), ("fp64", "direct"), ("bf16", "gmres"),
                                         ("fp32", "gmres")])
@pytest.mark.parametrize("m,n,p", [(150, 70, 12), (40, 40, 5), (60, 90, 40)])
def test_zlse_against_complex_oracle(h, prec, solver, m, n, p):
    note(f"zlse {prec} {solver} m={m} n={n} p={p}")
    rng = np.random.default_rng(3000 + m + n + p)
    A = conditioned_c(rng, m, n, 1e2)
    B, b, d = crandn(rng, p, n), crandn(rng, m), crandn(rng, p)
    x, r, v = lsq.empty_c(n), lsq.empty_c(m), lsq.empty_c(p)
    rc, res = h.zlse_solve(C(A), C(B), C(b), C(d), x, r, v, lsq.default_opts(prec=prec, solver=solver))
    assert rc == 0, (rc, h.last_error(), res.as_dict())
    assert res.berr_max <= 1e-14
    xg, rg, vg = H(x), H(r), H(v)
    be = zc.zlse_berr(A, B, b, d, xg, rg, vg)
    assert be[3] <= 1.01e-14
    xo, ro, vo = zc.zlse_solve(A, B, b, d)
    cond = zc.zlse_cond_x(A, B, xo, ro, vo)
    assert _rel(xg, xo) <= 10 * cond * U64
    assert zc.zlse_err1(B, d, xg) <= 1e-14


@pytest.mark.parametrize("prec,solver", [("fp32", "ir"), ("fp64", "direct"), ("fp32", "gmres")])
@pytest.mark.parametrize("n,m,p", [(120, 30, 100), (50, 50, 20), (90, 40, 60)])
def test_zgls_against_complex_oracle(h, prec, solver, n, m, p):
    note(f"zgls {prec} {solver} n={n} m={m} p={p}")
    rng = np.random.default_rng(4000 + n + m + p)
    W = crandn(rng, n, m)
    V = conditioned_c(rng, n, p, 1e2)
    d = crandn(rng, n)
    x, y, z = lsq.empty_c(m), lsq.empty_c(p), lsq.empty_c(n)
    rc, res = h.zgls_solve(C(W), C(V), C(d), x, y, z, lsq.default_opts(prec=prec, solver=solver))
    assert rc == 0, (rc, h.last_error(), res.as_dict())
    xg, yg, zg = H(x), H(y), H(z)
    be = zc.zgls_berr(W, V, d, xg, yg, zg)
    assert be[3] <= 1.01e-14
    xo, yo, zo = zc.zgls_solve(W, V, d)
    cx, cy = zc.zgls_cond_xy(W, V, xo, yo, zo)
    assert _rel(xg, xo) <= 10 * cx * U64
    if np.max(np.abs(yo)) > 0:
        assert _rel(yg, yo) <= 10 * cy * U64
    else:
        assert np.max(np.abs(yg)) <= 1e-14 * (np.linalg.norm(d) + 1)


def test_zlse_berr_is_that_of_the_complex_problem(h):
    # stopped after the initial solve (maxit 0, no escalation) the FP32
    # iterate's backward error is far above rounding level: the library's
    # figure equals the complex problem's (Frobenius norms of the complex
    # matrices), not the real embedding's (sqrt(2) times larger matrix norms)
    note("zlse berr of an unconverged iterate")
    rng = np.random.default_rng(3102)
    m, n, p = 120, 60, 10
    A = conditioned_c(rng, m, n, 1e4)
    B, b, d = crandn(rng, p, n), crandn(rng, m), crandn(rng, p)
    x, r, v = lsq.empty_c(n), lsq.empty_c(m), lsq.empty_c(p)
    rc, res = h.zlse_solve(C(A), C(B), C(b), C(d), x, r, v,
                           lsq.default_opts(prec="bf16", maxit=0, escalate=0))
    assert rc == 3, (rc, h.last_error(), res.as_dict())
    be = zc.zlse_berr(A, B, b, d, H(x), H(r), H(v))
    assert be[3] > 1e-6
    for q in range(3):
        assert abs(res.berr[q] - be[q]) <= 1e-6 * be[q] + 1e-300
    # the same blocks with the embedding's matrix norms differ by far more
    Ae = np.block([[A.real, -A.imag], [A.imag, A.real]])
    assert abs(np.linalg.norm(Ae) / np.linalg.norm(A) - np.sqrt(2)) <= 1e-12


def test_zlse_real_data_matches_real_solve(h):
    # real data through the complex entry point: the imaginary parts stay zero
    # and the solution equals that of the real entry point
    note("zlse with real data vs lse_solve")
    rng = np.random.default_rng(3100)
    P = wl.lse_conditioned(rng, 100, 50, 10, 1e2)
    m, n = P.A.shape
    p = P.B.shape[0]
    x, r, v = lsq.empty_c(n), lsq.empty_c(m), lsq.empty_c(p)
    rc, res = h.zlse_solve(C(P.A), C(P.B), C(P.b), C(P.d), x, r, v, lsq.default_opts(prec="fp32"))
    assert rc == 0
    xr = lsq.empty(n)
    rc2, _ = h.lse_solve(lsq.colmajor(P.A), lsq.colmajor(P.B), lsq.colmajor(P.b), lsq.colmajor(P.d),
                         xr, None, None, lsq.default_opts(prec="fp32"))
    assert rc2 == 0
    xg = H(x)
    assert np.max(np.abs(xg.imag)) <= 1e-13 * np.max(np.abs(xg))
    assert _rel(xg.real, H(xr)) <= 1e-12


def test_zlse_argument_checks(h):
    note("zlse argument checks")
    rng = np.random.default_rng(3101)
    A, B, b, d = crandn(rng, 10, 6), crandn(rng, 2, 6), crandn(rng, 10), crandn(rng, 2)
    x = lsq.empty_c(6)
    lib = h.lib
    rc = lib.zlse_solve(h.h, 10, 6, 7, lsq._cptr(C(A)), 10, lsq._cptr(C(B)), 2, lsq._cptr(C(b)),
                        lsq._cptr(C(d)), lsq._cptr(x), None, None, None, None)
    assert rc == -4
    rc = lib.zlse_solve(h.h, 10, 6, 2, lsq._cptr(C(A)), 9, lsq._cptr(C(B)), 2, lsq._cptr(C(b)),
                        lsq._cptr(C(d)), lsq._cptr(x), None, None, None, None)
    assert rc == -6
    bad = b.copy()
    bad[4] = complex(np.nan, 0)
    rc, res = h.zlse_solve(C(A), C(B), C(bad), C(d), x)
    assert rc == 5 and res.info == 5
