"""GMRES-IR on the GPU: the block-diagonal split-preconditioned operator and
end-to-end GMRES-IR solves, through the C-ABI, against the oracle and the
spectrum of Lemma C.1."""
import math
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
    hd = lsq.Handle()
    yield hd
    hd.close()


def D(a):
    return lsq.colmajor(a)


def H(t):
    return t.detach().cpu().numpy()


def rng(s):
    return np.random.default_rng(s)


def _assemble(h, kind, prec, A, B, alpha, beta, N):
    cols = []
    for e in np.eye(N):
        cols.append(H(h.dbg_bd_apply(kind, prec, D(A), D(B), alpha, beta, lsq.colmajor(e))))
    return np.column_stack(cols)


def _spectrum_counts(X, tol):
    """Eigenvalues of the symmetric part sorted into the clusters of Lemma
    C.1: 1, the golden-ratio pair (1 +- sqrt 5) / 2 and the roots of
    t^3 - t^2 - 2t + 1, plus -1, which the n > m (LSE) and n > p (GLS)
    preconditioners add: there the preconditioned matrix pairs n - m
    (n - p) entries of the x- (z-) block with the v- (x-) block alone, a
    [0 1; 1 0] block."""
    ev = np.sort(np.linalg.eigvalsh((X + X.T) / 2))
    phi = (1 + math.sqrt(5)) / 2
    cub = np.roots([1.0, -1.0, -2.0, 1.0]).real
    targets = {"one": [1.0], "minus_one": [-1.0], "golden": [phi, 1 - phi], "cubic": list(cub)}
    counts = {k: 0 for k in targets}
    for e in ev:
        hit = [k for k, vals in targets.items() if min(abs(e - t) for t in vals) < tol]
        assert len(hit) == 1, e
        counts[hit[0]] += 1
    return counts


@pytest.mark.parametrize("m,n,p,alpha,beta", [(30, 12, 4, 0.7, 1.3), (20, 20, 5, 1.0, 1.0), (70, 9, 9, 2.5, 0.4)])
def test_lse_bd_operator_spectrum_fp64(h, m, n, p, alpha, beta):
    note(f"lse bd operator m={m} n={n} p={p}")
    P = wl.lse_gaussian(rng(60 + m), m, n, p)
    N = m + n + p
    X = _assemble(h, "lse", "fp64", P.A, P.B, alpha, beta, N)
    assert np.max(np.abs(X - X.T)) < 1e-10 * np.max(np.abs(X))
    assert _spectrum_counts(X, 1e-8) == {"one": m - n, "minus_one": 0, "golden": 2 * (n - p),
                                         "cubic": 3 * p}


@pytest.mark.parametrize("m,n,p,alpha,beta", [(8, 12, 6, 0.8, 1.7), (40, 70, 45, 1.0, 1.0),
                                              (20, 36, 16, 2.2, 0.5), (50, 90, 70, 0.6, 1.1)])
def test_lse_bd_operator_spectrum_nlarge_fp64(h, m, n, p, alpha, beta):
    # eq. lse-bdpre-nlarge: n - m pairs with eigenvalues +-1, m - n + p cubic triples
    note(f"lse bd operator n>m m={m} n={n} p={p}")
    P = wl.lse_gaussian(rng(90 + m), m, n, p)
    N = m + n + p
    X = _assemble(h, "lse", "fp64", P.A, P.B, alpha, beta, N)
    assert np.max(np.abs(X - X.T)) < 1e-10 * np.max(np.abs(X))
    assert _spectrum_counts(X, 1e-8) == {"one": n - m, "minus_one": n - m, "golden": 2 * (n - p),
                                         "cubic": 3 * (m - n + p)}


@pytest.mark.parametrize("n,m,p,alpha,beta", [(12, 8, 6, 1.4, 0.5), (70, 40, 45, 1.0, 1.0),
                                              (36, 20, 16, 0.5, 2.2), (90, 50, 70, 1.1, 0.6)])
def test_gls_bd_operator_spectrum_nlarge_fp64(h, n, m, p, alpha, beta):
    # eq. gls-bdpre-nlarge: n - p pairs with eigenvalues +-1, n - m golden pairs
    note(f"gls bd operator n>p n={n} m={m} p={p}")
    G = wl.gls_gaussian(rng(92 + n), n, m, p)
    N = m + n + p
    X = _assemble(h, "gls", "fp64", G.W, G.V, alpha, beta, N)
    assert np.max(np.abs(X - X.T)) < 1e-10 * np.max(np.abs(X))
    assert _spectrum_counts(X, 1e-8) == {"one": n - p, "minus_one": n - p, "golden": 2 * (n - m),
                                         "cubic": 3 * (m - n + p)}


@pytest.mark.parametrize("n,m,p,alpha,beta", [(12, 4, 30, 1.9, 0.6), (16, 16, 16, 1.0, 1.0), (10, 3, 47, 0.3, 2.0)])
def test_gls_bd_operator_spectrum_fp64(h, n, m, p, alpha, beta):
    note(f"gls bd operator n={n} m={m} p={p}")
    G = wl.gls_gaussian(rng(62 + n), n, m, p)
    N = m + n + p
    X = _assemble(h, "gls", "fp64", G.W, G.V, alpha, beta, N)
    assert np.max(np.abs(X - X.T)) < 1e-10 * np.max(np.abs(X))
    assert _spectrum_counts(X, 1e-8) == {"one": p - n, "minus_one": 0, "golden": 2 * (n - m),
                                         "cubic": 3 * m}


def test_lse_bd_operator_fp32_near_clusters(h):
    # with FP32 factors the eigenvalues move by O(kappa u_f) from the clusters
    note("lse bd operator fp32")
    m, n, p = 40, 16, 5
    P = wl.lse_gaussian(rng(70), m, n, p)
    X = _assemble(h, "lse", "fp32", P.A, P.B, 0.9, 1.0, m + n + p)
    assert _spectrum_counts(X, 1e-3) == {"one": m - n, "minus_one": 0, "golden": 2 * (n - p),
                                         "cubic": 3 * p}


def _check_lse(P, x, r, v, res, tol=1e-14):
    assert res.berr_max <= tol
    be = direct.lse_berr(P.A, P.B, P.b, P.d, x, r, v)
    assert be[3] <= tol * 1.01
    xo, ro, vo = direct.lse_solve(P.A, P.B, P.b, P.d)
    cond = direct.lse_cond_x(P.A, P.B, xo, ro, vo)
    fwd = np.max(np.abs(x - xo)) / np.max(np.abs(xo))
    assert fwd <= 10 * cond * U64


def _fwd(a, ref):
    s = np.max(np.abs(ref)) if ref.size else 0.0
    d = np.max(np.abs(a - ref)) if ref.size else 0.0
    return d / s if s > 0 else d


def _check_gls(G, x, y, z, res, tol=1e-14):
    assert res.berr_max <= tol
    be = direct.gls_berr(G.W, G.V, G.d, x, y, z)
    assert be[3] <= tol * 1.01
    xo, yo, zo = direct.gls_solve(G.W, G.V, G.d)
    cx, cy = direct.gls_cond_xy(G.W, G.V, xo, yo, zo)
    assert _fwd(x, xo) <= 10 * cx * U64
    assert _fwd(y, yo) <= 10 * cy * U64


@pytest.mark.parametrize("prec,kappa", [("fp32", 1e3), ("fp32", 1e7), ("bf16", 1e2), ("fp16", 1e3)])
def test_lse_gmres_ir(h, prec, kappa):
    note(f"lse gmres-ir prec={prec} kappa={kappa:g}")
    P = wl.lse_paper_pair(rng(11), 512, 128, 8, kappa)
    m, n, p = P.shape
    x, r, v = lsq.empty(n), lsq.empty(m), lsq.empty(p)
    opts = lsq.default_opts(prec=prec, solver="gmres", escalate=0)
    rc, res = h.lse_solve(D(P.A), D(P.B), D(P.b), D(P.d), x, r, v, opts)
    assert rc == 0, (rc, h.last_error(), res.as_dict())
    d = res.as_dict()
    assert d["solver_used"] == "gmres" and d["prec_used"] == prec and d["attempts"] == 1
    assert 0 < res.gmres_iters <= 300
    _check_lse(P, H(x), H(r), H(v), res)


@pytest.mark.parametrize("prec,kappa", [("fp32", 1e3), ("fp32", 1e7), ("bf16", 1e2), ("fp16", 1e3)])
def test_gls_gmres_ir(h, prec, kappa):
    note(f"gls gmres-ir prec={prec} kappa={kappa:g}")
    G = wl.gls_paper_pair(rng(12), 128, 8, 512, kappa)
    n, m, p = G.shape
    x, y, z = lsq.empty(m), lsq.empty(p), lsq.empty(n)
    opts = lsq.default_opts(prec=prec, solver="gmres", escalate=0)
    rc, res = h.gls_solve(D(G.W), D(G.V), D(G.d), x, y, z, opts)
    assert rc == 0, (rc, h.last_error(), res.as_dict())
    d = res.as_dict()
    assert d["solver_used"] == "gmres" and d["prec_used"] == prec and d["attempts"] == 1
    _check_gls(G, H(x), H(y), H(z), res)


def test_gmres_ir_needs_fewer_outer_steps_than_classical(h):
    # the behaviour the paper reports for ill-conditioned pairs (Table 4)
    note("lse gmres vs classical kappa 1e7")
    P = wl.lse_paper_pair(rng(11), 512, 128, 8, 1e7)
    m, n, p = P.shape
    out = {}
    for solver in ("ir", "gmres"):
        x, r, v = lsq.empty(n), lsq.empty(m), lsq.empty(p)
        rc, res = h.lse_solve(D(P.A), D(P.B), D(P.b), D(P.d), x, r, v,
                              lsq.default_opts(prec="fp32", solver=solver, escalate=0, tol=1e-13))
        out[solver] = (rc, res.ir_steps)
    assert out["gmres"][0] == 0
    assert out["ir"][0] != 0 or out["gmres"][1] < out["ir"][1]


def test_gls_gmres_ir_config3_scaled(h):
    # the structure of the large GLS workload (W Gaussian, V = U diag(s) V^T
    # with kappa(V) = 1e6, n = p), at a quarter of its size
    note("gls gmres-ir config3 scaled 1024x256x1024 bf16")
    G = wl.config3(n=1024, m=256, p=1024)
    n, m, p = G.shape
    x, y, z = lsq.empty(m), lsq.empty(p), lsq.empty(n)
    rc, res = h.gls_solve(D(G.W), D(G.V), D(G.d), x, y, z,
                          lsq.default_opts(prec="bf16", solver="gmres"))
    assert rc == 0, (rc, h.last_error(), res.as_dict())
    assert res.berr_max <= 1e-14
    be = direct.gls_berr(G.W, G.V, G.d, H(x), H(y), H(z))
    assert be[3] <= 1.01e-14
    xo, yo, zo = direct.gls_solve(G.W, G.V, G.d)
    cx, cy = direct.gls_cond_xy_est(G.W, G.V, xo, yo, zo)
    assert _fwd(H(x), xo) <= 10 * cx * U64 and _fwd(H(y), yo) <= 10 * cy * U64


def test_ladder_escalates_from_bf16_ir(h):
    # kappa 1e6 is beyond BF16's reach for classical IR: the ladder moves on
    note("lse ladder bf16 kappa 1e6")
    P = wl.lse_paper_pair(rng(13), 256, 64, 8, 1e6)
    m, n, p = P.shape
    x, r, v = lsq.empty(n), lsq.empty(m), lsq.empty(p)
    rc, res = h.lse_solve(D(P.A), D(P.B), D(P.b), D(P.d), x, r, v,
                          lsq.default_opts(prec="bf16", solver="ir", escalate=1))
    assert rc == 0, (rc, h.last_error(), res.as_dict())
    assert res.attempts > 1
    _check_lse(P, H(x), H(r), H(v), res)


def test_gmres_request_on_lse_m_below_n_runs_gmres(h):
    # LSE with m < n uses eq. lse-bdpre-nlarge
    note("lse m<n gmres request")
    P = wl.lse_gaussian(rng(14), 20, 30, 15)
    m, n, p = P.shape
    x, r, v = lsq.empty(n), lsq.empty(m), lsq.empty(p)
    rc, res = h.lse_solve(D(P.A), D(P.B), D(P.b), D(P.d), x, r, v,
                          lsq.default_opts(prec="fp32", solver="gmres", escalate=0))
    assert rc == 0 and res.as_dict()["solver_used"] == "gmres" and res.gmres_iters > 0
    _check_lse(P, H(x), H(r), H(v), res)


# The preconditioned matrix is X - dE with ||dE|| = O(u_f) kappa(A) kappa(B)
# (Section 5.2); the BF16 cases keep u_f kappa(A) kappa(B) ~ 0.1, below the
# smallest singular value 0.445 of X, with both matrices conditioned.
@pytest.mark.parametrize("prec,kappa,shape", [("fp32", 1e3, (300, 420, 200)), ("fp32", 1e6, (130, 160, 64)),
                                              ("bf16", 5.0, (380, 420, 64)), ("fp32", 1e4, (64, 127, 64))])
def test_lse_gmres_ir_nlarge(h, prec, kappa, shape):
    # n > m: several 64-column panels and a ragged tail; n = m + p - 1 at the
    # last case (at n = m + p the exact r and v vanish and the third block of
    # the stop test compares rounding errors with rounding errors)
    m, n, p = shape
    note(f"lse gmres-ir n>m prec={prec} kappa={kappa:g} m={m} n={n} p={p}")
    kb = 5.0 if prec == "bf16" else None
    P = wl.lse_conditioned(rng(int(kappa) % 97 + m), m, n, p, kappa, kb)
    x, r, v = lsq.empty(n), lsq.empty(m), lsq.empty(p)
    rc, res = h.lse_solve(D(P.A), D(P.B), D(P.b), D(P.d), x, r, v,
                          lsq.default_opts(prec=prec, solver="gmres", escalate=0))
    assert rc == 0, (rc, h.last_error(), res.as_dict())
    d = res.as_dict()
    assert d["solver_used"] == "gmres" and d["prec_used"] == prec and d["attempts"] == 1
    assert 0 < res.gmres_iters <= 300
    _check_lse(P, H(x), H(r), H(v), res)


@pytest.mark.parametrize("prec,kappa,shape", [("fp32", 1e3, (420, 300, 200)), ("fp32", 1e5, (160, 130, 64)),
                                              ("bf16", 5.0, (420, 380, 64)), ("fp32", 1e4, (128, 64, 64))])
def test_gls_gmres_ir_nlarge(h, prec, kappa, shape):
    # n > p: several panels and a ragged tail; n = m + p at the last case
    n, m, p = shape
    note(f"gls gmres-ir n>p prec={prec} kappa={kappa:g} n={n} m={m} p={p}")
    kw = 5.0 if prec == "bf16" else None
    G = wl.gls_conditioned(rng(int(kappa) % 89 + n), n, m, p, kappa, kw)
    x, y, z = lsq.empty(m), lsq.empty(p), lsq.empty(n)
    rc, res = h.gls_solve(D(G.W), D(G.V), D(G.d), x, y, z,
                          lsq.default_opts(prec=prec, solver="gmres", escalate=0))
    assert rc == 0, (rc, h.last_error(), res.as_dict())
    d = res.as_dict()
    assert d["solver_used"] == "gmres" and d["prec_used"] == prec and d["attempts"] == 1
    assert 0 < res.gmres_iters <= 300
    _check_gls(G, H(x), H(y), H(z), res)


def test_lse_gmres_ir_nlarge_matches_oracle_iteration(h):
    # the same GMRES-IR on the CPU (FP32 factors, FP64 GMRES) and on the GPU:
    # both certify, and both land on the oracle's direct solution
    from oracle import mpir
    note("lse gmres-ir n>m vs oracle mplse_gmres_bd")
    P = wl.lse_conditioned(rng(15), 96, 128, 48, 1e5)
    m, n, p = P.shape
    g = mpir.mplse_gmres_bd(P.A, P.B, P.b, P.d, tol=1e-14)
    assert g.converged
    x, r, v = lsq.empty(n), lsq.empty(m), lsq.empty(p)
    rc, res = h.lse_solve(D(P.A), D(P.B), D(P.b), D(P.d), x, r, v,
                          lsq.default_opts(prec="fp32", solver="gmres", escalate=0))
    assert rc == 0, (rc, h.last_error(), res.as_dict())
    _check_lse(P, H(x), H(r), H(v), res)
    assert _fwd(H(x), g.x) <= 1e-10


@pytest.mark.parametrize("kind,shape", [("lse", (300, 120, 20)), ("gls", (150, 40, 260)),
                                        ("lse", (120, 200, 100)), ("gls", (200, 120, 100))])
def test_bd_operator_graph_replays_match_eager(h, kind, shape):
    # the GMRES operator is captured once as a HIP graph and replayed: every
    # replay (with eager copies in between) must equal the eager application
    note(f"bd operator graph replays {kind} {shape}")
    if kind == "lse":
        P = wl.lse_gaussian(rng(80), *shape)
        A, B = P.A, P.B
        N = sum(P.shape)
    else:
        G = wl.gls_gaussian(rng(81), *shape)
        A, B = G.W, G.V
        N = sum(G.shape)
    U = rng(82).standard_normal((N, 4))
    Y, used = h.dbg_bd_apply_graph(kind, "fp32", D(A), D(B), 0.8, 1.0, D(U))
    assert used
    Y = H(Y)
    for j in range(U.shape[1]):
        ref = H(h.dbg_bd_apply(kind, "fp32", D(A), D(B), 0.8, 1.0, lsq.colmajor(U[:, j])))
        assert np.max(np.abs(Y[:, j] - ref)) <= 1e-12 * (1 + np.max(np.abs(ref)))
