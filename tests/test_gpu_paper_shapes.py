"""The paper's experiment shapes (Section 6: LSE with m > n >> p and m >> n > p,
GLS with p > n >> m), scaled down, on the GPU: FP32 factorization with
classical IR and with GMRES-IR (escalation on) must certify berr <= 1e-14 and
land on the oracle's FP64 solution within the conditioning bound."""
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


def H(t):
    return t.detach().cpu().numpy()


def _fwd(a, ref):
    s = np.max(np.abs(ref)) if ref.size else 0.0
    d = np.max(np.abs(a - ref)) if ref.size else 0.0
    return d / s if s > 0 else d


# (experiment, n, m / n, n / p) for LSE; kappa of the stacked [A^T, B^T]
LSE_CASES = [("E1", 256, 8, 32, 1e3), ("E1", 256, 12, 64, 1e7), ("E2", 32, 128, 8, 1e5)]
# (experiment, n, p / n, n / m) for GLS; kappa of [W, V]
GLS_CASES = [("E3", 256, 8, 32, 1e3), ("E3", 256, 12, 64, 1e7)]


@pytest.mark.parametrize("solver", ["ir", "gmres"])
@pytest.mark.parametrize("exp,n,fm,fp,kappa", LSE_CASES)
def test_lse_paper_shapes(h, exp, n, fm, fp, kappa, solver):
    m, p = fm * n, n // fp
    note(f"{exp} lse m={m} n={n} p={p} kappa={kappa:g} solver={solver}")
    P = wl.lse_paper_pair(np.random.default_rng(int(np.log10(kappa)) * 7 + n), m, n, p, kappa)
    x, r, v = lsq.empty(n), lsq.empty(m), lsq.empty(p)
    rc, res = h.lse_solve(lsq.colmajor(P.A), lsq.colmajor(P.B), lsq.colmajor(P.b), lsq.colmajor(P.d),
                          x, r, v, lsq.default_opts(prec="fp32", solver=solver, escalate=1))
    assert rc == 0, (rc, h.last_error(), res.as_dict())
    assert res.berr_max <= 1e-14
    be = direct.lse_berr(P.A, P.B, P.b, P.d, H(x), H(r), H(v))
    assert be[3] <= 1.01e-14
    xo, ro, vo = direct.lse_solve(P.A, P.B, P.b, P.d)
    cond = direct.lse_cond_x(P.A, P.B, xo, ro, vo)
    assert _fwd(H(x), xo) <= 10 * cond * U64


@pytest.mark.parametrize("solver", ["ir", "gmres"])
@pytest.mark.parametrize("exp,n,fpn,fnm,kappa", GLS_CASES)
def test_gls_paper_shapes(h, exp, n, fpn, fnm, kappa, solver):
    p, m = fpn * n, n // fnm
    note(f"{exp} gls n={n} m={m} p={p} kappa={kappa:g} solver={solver}")
    G = wl.gls_paper_pair(np.random.default_rng(int(np.log10(kappa)) * 7 + n + 1), n, m, p, kappa)
    x, y, z = lsq.empty(m), lsq.empty(p), lsq.empty(n)
    rc, res = h.gls_solve(lsq.colmajor(G.W), lsq.colmajor(G.V), lsq.colmajor(G.d), x, y, z,
                          lsq.default_opts(prec="fp32", solver=solver, escalate=1))
    assert rc == 0, (rc, h.last_error(), res.as_dict())
    assert res.berr_max <= 1e-14
    be = direct.gls_berr(G.W, G.V, G.d, H(x), H(y), H(z))
    assert be[3] <= 1.01e-14
    xo, yo, zo = direct.gls_solve(G.W, G.V, G.d)
    cx, cy = direct.gls_cond_xy(G.W, G.V, xo, yo, zo)
    assert _fwd(H(x), xo) <= 10 * cx * U64
    assert _fwd(H(y), yo) <= 10 * cy * U64
