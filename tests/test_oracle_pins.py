"""Pins of the oracle's stop-test scales, backward errors, err-1 / err-2,
assumption checks and block condition numbers.

The expected values come from outside the oracle:
- a hand-worked LSE and GLS with small integer data, whose solutions,
  residual blocks, scales (eq. lse-stop, eq. gls-stop), backward errors and
  err-1 / err-2 (Tables 4 and 5) are written out with their derivations in
  tests/golden/hand_worked_lse_gls.txt;
- exact rational arithmetic (sympy) for ranks and for the Skeel condition
  numbers of the augmented systems of those instances.

Each group also carries planted mistakes (a spectral norm where the
Frobenius norm belongs, a dropped term, a wrong block slice) and checks that
the golden values reject them.
"""
import os

import numpy as np
import pytest
import sympy

from oracle import direct

GOLD = os.path.join(os.path.dirname(__file__), "golden", "hand_worked_lse_gls.txt")


def _gold():
    out = {}
    with open(GOLD) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#") or "=" not in line:
                continue
            k, v = line.split("=", 1)
            out[k.strip()] = float(v)
    return out


G = _gold()

# the hand-worked instances (see the golden file)
A = np.array([[1.0, 0.0], [0.0, 1.0], [1.0, 1.0]])
B = np.array([[1.0, 1.0]])
b = np.array([1.0, 2.0, 3.0])
d = np.array([1.0])
XH, RH, VH = np.array([1.0, 1.0]), np.array([0.0, 0.0, 1.0]), np.array([2.0])

W = np.array([[1.0], [1.0]])
V = np.array([[1.0, 0.0], [0.0, 2.0]])
dg = np.array([2.0, 0.0])
XG, YG, ZG = np.array([1.0]), np.array([1.0, 0.0]), np.array([2.0, -1.0])

TOL = 4e-16


def _vec(prefix, n):
    return np.array([G[f"{prefix}{i}"] for i in range(n)])


# ------------------------------------------------------------- solutions --

def test_hand_lse_solution():
    x, r, v = direct.lse_solve(A, B, b, d)
    assert np.allclose(x, _vec("lse.x", 2), rtol=0, atol=1e-15)
    assert np.allclose(r, _vec("lse.r", 3), rtol=0, atol=1e-15)
    assert np.allclose(v, _vec("lse.v", 1), rtol=0, atol=1e-14)


def test_hand_gls_solution():
    x, y, z = direct.gls_solve(W, V, dg)
    assert np.allclose(x, _vec("gls.x", 1), rtol=0, atol=1e-15)
    assert np.allclose(y, _vec("gls.y", 2), rtol=0, atol=1e-15)
    assert np.allclose(z, _vec("gls.z", 2), rtol=0, atol=1e-15)


# ---------------------------------------- residual, scales, backward error --

def test_hand_lse_residual_scales_berr():
    f1, f2, f3 = direct.lse_residual(A, B, b, d, XH, RH, VH)
    assert np.array_equal(f1, _vec("lse.f1_", 3))
    assert np.array_equal(f2, _vec("lse.f2_", 1))
    assert np.array_equal(f3, _vec("lse.f3_", 2))
    s = direct.lse_scales(A, B, b, d, XH, RH, VH)
    for i in range(3):
        assert s[i] == pytest.approx(G[f"lse.scale{i + 1}"], rel=TOL)
    e = direct.lse_berr(A, B, b, d, XH, RH, VH)
    for i in range(3):
        assert e[i] == pytest.approx(G[f"lse.berr{i + 1}"], rel=TOL)
    assert e[3] == max(e[:3])


def test_hand_gls_residual_scales_berr():
    f1, f2, f3 = direct.gls_residual(W, V, dg, XG, YG, ZG)
    assert np.array_equal(f1, _vec("gls.f1_", 2))
    assert np.array_equal(f2, _vec("gls.f2_", 2))
    assert np.array_equal(f3, _vec("gls.f3_", 1))
    s = direct.gls_scales(W, V, dg, XG, YG, ZG)
    for i in range(3):
        assert s[i] == pytest.approx(G[f"gls.scale{i + 1}"], rel=TOL)
    e = direct.gls_berr(W, V, dg, XG, YG, ZG)
    for i in range(3):
        assert e[i] == pytest.approx(G[f"gls.berr{i + 1}"], rel=TOL)
    assert e[3] == max(e[:3])


def test_berr_is_zero_at_the_exact_hand_solutions():
    x, r, v = direct.lse_solve(A, B, b, d)
    assert direct.lse_berr(A, B, b, d, x, r, v)[3] <= 1e-15
    x, y, z = direct.gls_solve(W, V, dg)
    assert direct.gls_berr(W, V, dg, x, y, z)[3] <= 1e-15


def _spectral(M):
    return float(np.linalg.norm(M, 2)) if M.size else 0.0


def test_planted_spectral_norm_in_the_scales_is_rejected(monkeypatch):
    # the stop tests use Frobenius norms of the matrices; with the spectral
    # norm in their place (sqrt(3) for A, 2 for V) the golden scales fail
    monkeypatch.setattr(direct, "_fro", _spectral)
    s = direct.lse_scales(A, B, b, d, XH, RH, VH)
    assert s[0] != pytest.approx(G["lse.scale1"], rel=1e-6)
    assert s[2] != pytest.approx(G["lse.scale3"], rel=1e-6)
    s = direct.gls_scales(W, V, dg, XG, YG, ZG)
    assert s[0] != pytest.approx(G["gls.scale1"], rel=1e-6)
    assert s[1] != pytest.approx(G["gls.scale2"], rel=1e-6)


def test_planted_dropped_terms_are_rejected():
    # each term of each scale is nonzero in the hand-worked iterates, so
    # dropping any one of them moves the value away from the golden one
    nA, nB, nW, nV = 2.0, np.sqrt(2.0), np.sqrt(2.0), np.sqrt(5.0)
    nb, nd, nx, nr, nv = np.sqrt(14.0), 1.0, np.sqrt(2.0), 1.0, 2.0
    lse_terms = [(nb, nr, nA * nx), (nd, nB * nx), (nA * nr, nB * nv)]
    nd_, nxg, nyg, nzg = 2.0, 1.0, 1.0, np.sqrt(5.0)
    gls_terms = [(nyg, nV * nzg), (nd_, nW * nxg, nV * nyg), (nW * nzg,)]
    for name, terms in (("lse", lse_terms), ("gls", gls_terms)):
        for i, t in enumerate(terms):
            full = sum(t)
            assert full == pytest.approx(G[f"{name}.scale{i + 1}"], rel=1e-15)
            for j in range(len(t)):
                assert full - t[j] != pytest.approx(G[f"{name}.scale{i + 1}"], rel=1e-6)


# ------------------------------------------------------------ err-1, err-2 --

def test_hand_err1_err2():
    x, _, _ = direct.lse_solve(A, B, b, d)
    assert direct.lse_err1(B, d, XH) == pytest.approx(G["lse.err1"], rel=TOL)
    assert direct.lse_err2(A, b, XH, x) == pytest.approx(G["lse.err2"], rel=1e-14)
    xg, yg, _ = direct.gls_solve(W, V, dg)
    assert direct.gls_err1(W, V, dg, XG, YG) == pytest.approx(G["gls.err1"], rel=TOL)
    assert direct.gls_err2(YG, yg) == pytest.approx(G["gls.err2"], rel=1e-14)
    # at the exact solutions both metrics are at rounding level
    assert direct.lse_err1(B, d, x) <= 1e-15 and direct.lse_err2(A, b, x, x) == 0.0
    assert direct.gls_err1(W, V, dg, xg, yg) <= 1e-15 and direct.gls_err2(yg, yg) == 0.0


def test_planted_err_variants_are_rejected():
    # err-1 without the ||d|| term, err-2 without the "- 1", or the ratio
    # inverted: each differs from the golden value of the hand-worked case
    x = np.array([0.0, 1.0])
    nrm = np.linalg.norm
    assert nrm(B @ XH - d) / (np.sqrt(2.0) * nrm(XH)) != pytest.approx(G["lse.err1"], rel=1e-6)
    ratio = nrm(A @ XH - b) / nrm(A @ x - b)
    assert ratio != pytest.approx(G["lse.err2"], rel=1e-6)
    assert abs(1.0 / ratio - 1.0) != pytest.approx(G["lse.err2"], rel=1e-6)
    yref = np.array([0.4, -0.8])
    assert abs(nrm(yref) / nrm(YG) - 1.0) != pytest.approx(G["gls.err2"], rel=1e-6)


# ------------------------------------------------------ assumption checks --

def _aug_rank_exact(F):
    return sympy.Matrix([[sympy.Rational(str(v)) for v in row] for row in F]).rank()


LSE_CASES = {
    # name: (A, B, holds)
    "generic": (np.array([[1, 0, 2], [0, 1, 1], [1, 1, 0], [2, 0, 1]], float),
                np.array([[1, 1, 1]], float), True),
    "rank_B_deficient": (np.array([[1, 0, 2], [0, 1, 1], [1, 1, 0], [2, 0, 1]], float),
                         np.array([[1, 1, 1], [2, 2, 2]], float), False),
    "stack_rank_deficient": (np.array([[1, 1, 2], [0, 0, 1], [3, 3, 0], [2, 2, 1]], float),
                             np.array([[1, 1, 1]], float), False),
    "square_B": (np.array([[1, 0], [0, 1]], float), np.array([[1, 2], [3, 4]], float), True),
}


@pytest.mark.parametrize("name", sorted(LSE_CASES))
def test_lse_assumption_check_agrees_with_exact_ranks(name):
    A_, B_, holds = LSE_CASES[name]
    assert bool(direct.check_lse_assumptions(A_, B_)) is holds
    # the assumptions hold exactly when the augmented matrix is nonsingular
    F = direct.lse_augmented(A_, B_)
    assert (_aug_rank_exact(F) == F.shape[0]) is holds


def test_lse_assumption_check_rejects_shapes():
    # p > n and n > m + p violate p <= n <= m + p
    assert not direct.check_lse_assumptions(np.ones((3, 1)), np.array([[1.0], [2.0]]))
    assert not direct.check_lse_assumptions(np.array([[1.0, 0.0, 0.0]]), np.array([[0.0, 1.0, 0.0]]))


GLS_CASES = {
    "generic": (np.array([[1, 0], [0, 1], [1, 1]], float), np.array([[1, 2], [0, 1], [1, 0]], float), True),
    "rank_W_deficient": (np.array([[1, 2], [1, 2], [1, 2]], float),
                         np.array([[1, 2], [0, 1], [1, 0]], float), False),
    "stack_rank_deficient": (np.array([[1, 0], [0, 1], [0, 0]], float),
                             np.array([[1, 2], [0, 1], [0, 0]], float), False),
    "square_W": (np.array([[2, 1], [1, 1]], float), np.array([[1], [0]], float), True),
}


@pytest.mark.parametrize("name", sorted(GLS_CASES))
def test_gls_assumption_check_agrees_with_exact_ranks(name):
    W_, V_, holds = GLS_CASES[name]
    assert bool(direct.check_gls_assumptions(W_, V_)) is holds
    F = direct.gls_augmented(W_, V_)
    assert (_aug_rank_exact(F) == F.shape[0]) is holds


def test_gls_assumption_check_rejects_shapes():
    # m > n and n > m + p violate m <= n <= m + p
    assert not direct.check_gls_assumptions(np.ones((1, 2)), np.ones((1, 1)))
    assert not direct.check_gls_assumptions(np.ones((4, 1)), np.ones((4, 2)))


# --------------------------------------------------- block condition numbers --

def _exact_skeel_blocks(F, u, blocks):
    """|| (|F^-1| |F| |u|)[blk] ||_inf / || u[blk] ||_inf for each block, in
    exact rational arithmetic."""
    Fs = sympy.Matrix([[sympy.Rational(str(v)) for v in row] for row in F])
    us = sympy.Matrix([sympy.Rational(str(v)) for v in u])
    Fi = Fs.inv()
    t = Fi.applyfunc(abs) * (Fs.applyfunc(abs) * us.applyfunc(abs))
    out = []
    for lo, hi in blocks:
        num = max(t[i] for i in range(lo, hi))
        den = max(abs(us[i]) for i in range(lo, hi))
        out.append(float(num / den))
    return out


def test_lse_cond_x_takes_the_x_block():
    m, n, p = 3, 2, 1
    x, r, v = np.array([0.0, 1.0]), np.array([1.0, 1.0, 2.0]), np.array([3.0])
    u = np.concatenate([r, -v, x])
    ex = _exact_skeel_blocks(direct.lse_augmented(A, B), u, [(0, m), (m, m + p), (m + p, m + p + n)])
    got = direct.lse_cond_x(A, B, x, r, v)
    assert got == pytest.approx(ex[2], rel=1e-12)
    # the other blocks' values differ, so a wrong slice would be caught
    assert all(abs(e - ex[2]) > 1e-3 * ex[2] for e in ex[:2])


def test_gls_cond_xy_take_the_x_and_y_blocks():
    n, m, p = 2, 1, 2
    x, y, z = np.array([1.6]), np.array([0.4, -0.8]), np.array([0.4, -0.4])
    u = np.concatenate([y, -z, x])
    ex = _exact_skeel_blocks(direct.gls_augmented(W, V), u, [(0, p), (p, p + n), (p + n, p + n + m)])
    cx, cy = direct.gls_cond_xy(W, V, x, y, z)
    assert cx == pytest.approx(ex[2], rel=1e-12)
    assert cy == pytest.approx(ex[0], rel=1e-12)
    assert abs(ex[0] - ex[2]) > 1e-3 * ex[2] and abs(ex[1] - ex[2]) > 1e-3 * ex[2]
    assert abs(ex[1] - ex[0]) > 1e-3 * ex[0]


# ------------------------------------------------ condition-number estimate --

@pytest.mark.parametrize("m,n,p", [(200, 100, 20), (60, 30, 8), (30, 12, 4), (40, 40, 10)])
def test_lse_cond_estimate_brackets_the_dense_value(m, n, p):
    # the block 1-norm estimator gives a lower bound that is close to the
    # exact value computed with the dense inverse
    from paper_2406_16499_amd import workloads as wl
    P = wl.lse_gaussian(np.random.default_rng(m + n + p), m, n, p)
    x, r, v = direct.lse_solve(P.A, P.B, P.b, P.d)
    exact = direct.lse_cond_x(P.A, P.B, x, r, v)
    est = direct.lse_cond_x_est(P.A, P.B, x, r, v)
    assert 0.5 * exact <= est <= exact * (1 + 1e-10)


def test_gls_cond_estimate_brackets_the_dense_value():
    from paper_2406_16499_amd import workloads as wl
    G = wl.gls_gaussian(np.random.default_rng(3), 60, 20, 80)
    x, y, z = direct.gls_solve(G.W, G.V, G.d)
    ex = direct.gls_cond_xy(G.W, G.V, x, y, z)
    es = direct.gls_cond_xy_est(G.W, G.V, x, y, z)
    for e, c in zip(es, ex):
        assert 0.5 * c <= e <= c * (1 + 1e-10)


def test_cond_estimate_on_the_hand_worked_lse():
    # exact rational value of the x-block (see test_lse_cond_x_takes_the_x_block)
    m, n, p = 3, 2, 1
    x, r, v = np.array([0.0, 1.0]), np.array([1.0, 1.0, 2.0]), np.array([3.0])
    u = np.concatenate([r, -v, x])
    ex = _exact_skeel_blocks(direct.lse_augmented(A, B), u, [(m + p, m + p + n)])[0]
    assert direct.lse_cond_x_est(A, B, x, r, v) == pytest.approx(ex, rel=1e-12)
