"""CPU pins of the complex oracle (oracle/complex_lsq.py): each result is
checked against something other than the oracle's own formulas -- the dense
complex KKT system solved by LAPACK, closed forms, special cases that reduce
to textbook routines, the real oracle on real data, invariants, and a
hand-worked instance for the stop-test scales."""
import numpy as np
import pytest
import scipy.linalg as sla

from oracle import complex_lsq as zc
from oracle import direct

U = 2.0 ** -53


def crandn(rng, *shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def _rel(a, b):
    s = np.max(np.abs(b))
    return np.max(np.abs(a - b)) / s if s > 0 else np.max(np.abs(a))


@pytest.mark.parametrize("m,n,p", [(12, 7, 3), (9, 9, 2), (6, 8, 3), (15, 6, 0), (5, 4, 4)])
def test_zlse_matches_dense_kkt(m, n, p):
    rng = np.random.default_rng(1000 + m + 10 * n + 100 * p)
    A, B, b, d = crandn(rng, m, n), crandn(rng, p, n), crandn(rng, m), crandn(rng, p)
    x, r, v = zc.zlse_solve(A, B, b, d)
    F = zc.zlse_augmented(A, B)
    u = np.linalg.solve(F, np.concatenate([b, d, np.zeros(n)]))
    assert _rel(x, u[m + p:]) <= 1e-12
    assert _rel(r, u[:m]) <= 1e-12
    if p:
        assert _rel(v, -u[m:m + p]) <= 1e-12


def test_zlse_special_cases():
    rng = np.random.default_rng(1001)
    # p = 0: plain complex least squares
    A, b = crandn(rng, 20, 6), crandn(rng, 20)
    x, _, _ = zc.zlse_solve(A, np.zeros((0, 6)), b, np.zeros(0))
    assert _rel(x, np.linalg.lstsq(A, b, rcond=None)[0]) <= 1e-13
    # n = p: x = B^-1 d whatever A and b are
    B, d = crandn(rng, 5, 5), crandn(rng, 5)
    x, _, _ = zc.zlse_solve(crandn(rng, 8, 5), B, crandn(rng, 8), d)
    assert _rel(x, np.linalg.solve(B, d)) <= 1e-12


def test_zlse_real_data_reduces_to_real_oracle():
    rng = np.random.default_rng(1002)
    A, B = rng.standard_normal((14, 8)), rng.standard_normal((3, 8))
    b, d = rng.standard_normal(14), rng.standard_normal(3)
    xz, rz, vz = zc.zlse_solve(A, B, b, d)
    x, r, v = direct.lse_solve(A, B, b, d)
    assert np.max(np.abs(xz.imag)) <= 1e-14 and _rel(xz.real, x) <= 1e-12
    assert _rel(rz.real, r) <= 1e-12 and _rel(vz.real, v) <= 1e-11


def test_zlse_kkt_invariants():
    rng = np.random.default_rng(1003)
    m, n, p = 30, 12, 4
    A, B, b, d = crandn(rng, m, n), crandn(rng, p, n), crandn(rng, m), crandn(rng, p)
    x, r, v = zc.zlse_solve(A, B, b, d)
    assert np.linalg.norm(B @ x - d) <= 50 * U * (np.linalg.norm(B) * np.linalg.norm(x) + np.linalg.norm(d))
    # optimality: A^H (Ax - b) lies in range(B^H), i.e. is orthogonal to null(B)
    N = sla.null_space(B)
    g = A.conj().T @ (A @ x - b)
    assert np.linalg.norm(N.conj().T @ g) <= 1e-12 * np.linalg.norm(A) ** 2 * np.linalg.norm(x)
    # the multiplier: A^H r = B^H v
    assert np.linalg.norm(A.conj().T @ r - B.conj().T @ v) <= 1e-12 * np.linalg.norm(A) * np.linalg.norm(r)


@pytest.mark.parametrize("n,m,p", [(12, 4, 10), (8, 8, 3), (10, 3, 7), (9, 4, 9)])
def test_zgls_matches_dense_kkt(n, m, p):
    rng = np.random.default_rng(2000 + n + 10 * m + 100 * p)
    W, V, d = crandn(rng, n, m), crandn(rng, n, p), crandn(rng, n)
    x, y, z = zc.zgls_solve(W, V, d)
    F = zc.zgls_augmented(W, V)
    u = np.linalg.solve(F, np.concatenate([np.zeros(p), d, np.zeros(m)]))
    # relative to the whole solution (y = 0 exactly when n = m)
    s = np.max(np.abs(u))
    assert np.max(np.abs(y - u[:p])) <= 1e-12 * s
    assert np.max(np.abs(z + u[p:p + n])) <= 1e-12 * s
    assert np.max(np.abs(x - u[p + n:])) <= 1e-12 * s


def test_zgls_closed_forms():
    rng = np.random.default_rng(2001)
    n, m = 10, 4
    W, d = crandn(rng, n, m), crandn(rng, n)
    # square nonsingular V: weighted least squares with Omega = (V V^H)^-1
    V = crandn(rng, n, n)
    x, y, _ = zc.zgls_solve(W, V, d)
    Om = np.linalg.inv(V @ V.conj().T)
    xw = np.linalg.solve(W.conj().T @ Om @ W, W.conj().T @ Om @ d)
    assert _rel(x, xw) <= 1e-11
    assert _rel(y, np.linalg.solve(V, d - W @ x)) <= 1e-11
    # V = I: ordinary least squares, y the residual
    x, y, _ = zc.zgls_solve(W, np.eye(n), d)
    xo = np.linalg.lstsq(W, d, rcond=None)[0]
    assert _rel(x, xo) <= 1e-12 and _rel(y, d - W @ xo) <= 1e-12
    # n = m: y = 0, x = W^-1 d
    Ws = crandn(rng, 6, 6)
    x, y, _ = zc.zgls_solve(Ws, crandn(rng, 6, 3), d[:6])
    assert np.max(np.abs(y)) <= 1e-13 and _rel(x, np.linalg.solve(Ws, d[:6])) <= 1e-12


def test_zgls_real_data_reduces_to_real_oracle():
    rng = np.random.default_rng(2002)
    W, V, d = rng.standard_normal((11, 4)), rng.standard_normal((11, 9)), rng.standard_normal(11)
    xz, yz, zz = zc.zgls_solve(W, V, d)
    x, y, z = direct.gls_solve(W, V, d)
    assert _rel(xz.real, x) <= 1e-12 and _rel(yz.real, y) <= 1e-12 and _rel(zz.real, z) <= 1e-11
    assert max(np.max(np.abs(xz.imag)), np.max(np.abs(yz.imag))) <= 1e-13


def test_zlse_scales_hand_worked():
    # m = 2, n = 1, p = 1: A = [1 + i; 1], B = [i], b = [1; i], d = [2i].
    # Constraint: i x = 2i gives x = 2, so r = b - A x = [1 - 2 - 2i; i - 2]
    # = [-1 - 2i; -2 + i], ||r|| = sqrt(5 + 5) = sqrt(10).  At the iterate
    # x = 1, r = 0, v = 0: f1 = b - A = [-i; -1 + i] (norm sqrt(3)),
    # f2 = d - B x = 2i - i = i (norm 1), f3 = 0.  ||A||_F = sqrt(3),
    # ||B||_F = 1, ||b|| = sqrt(2), ||d|| = 2, so the scales are
    # sqrt(2) + sqrt(3), 2 + 1 and 0.
    A = np.array([[1 + 1j], [1]])
    B = np.array([[1j]])
    b = np.array([1, 1j])
    d = np.array([2j])
    x, r, v = zc.zlse_solve(A, B, b, d)
    assert abs(x[0] - 2) <= 1e-15
    assert np.allclose(r, [-1 - 2j, -2 + 1j], atol=1e-15, rtol=0)
    s = zc.zlse_scales(A, B, b, d, np.array([1.0 + 0j]), np.zeros(2, complex), np.zeros(1, complex))
    assert abs(s[0] - (np.sqrt(2) + np.sqrt(3))) <= 1e-15
    assert abs(s[1] - 3.0) <= 1e-15 and s[2] == 0.0
    e = zc.zlse_berr(A, B, b, d, np.array([1.0 + 0j]), np.zeros(2, complex), np.zeros(1, complex))
    assert abs(e[0] - np.sqrt(3) / (np.sqrt(2) + np.sqrt(3))) <= 1e-15
    assert abs(e[1] - 1.0 / 3.0) <= 1e-15 and e[2] == 0.0
    # a planted mistake, the Frobenius norm of the real embedding (sqrt(2) ||A||_F),
    # gives another first block
    assert abs(np.sqrt(3) / (np.sqrt(2) + np.sqrt(6)) - e[0]) > 0.05
    # at the solution the backward error is at rounding level
    assert zc.zlse_berr(A, B, b, d, x, r, v)[3] <= 4 * U


def test_zcond_and_errs():
    rng = np.random.default_rng(2003)
    A, B, b, d = crandn(rng, 8, 5), crandn(rng, 2, 5), crandn(rng, 8), crandn(rng, 2)
    x, r, v = zc.zlse_solve(A, B, b, d)
    c = zc.zlse_cond_x(A, B, x, r, v)
    assert c >= 1.0
    # the Skeel number is at most the normwise condition of F (inf-norm)
    F = zc.zlse_augmented(A, B)
    kinf = np.linalg.norm(F, np.inf) * np.linalg.norm(np.linalg.inv(F), np.inf)
    u = np.concatenate([r, -v, x])
    assert c <= kinf * np.max(np.abs(u)) / np.max(np.abs(x)) * (1 + 1e-12)
    assert zc.zlse_err1(B, d, x) <= 10 * U
    assert zc.zlse_err2(A, b, x, x) == 0.0
    W, V, dd = crandn(rng, 9, 3), crandn(rng, 9, 7), crandn(rng, 9)
    xg, yg, zg = zc.zgls_solve(W, V, dd)
    assert zc.zgls_err1(W, V, dd, xg, yg) <= 10 * U and zc.zgls_err2(yg, yg) == 0.0
    cx, cy = zc.zgls_cond_xy(W, V, xg, yg, zg)
    assert cx >= 1.0 and cy >= 1.0
    assert zc.zgls_berr(W, V, dd, xg, yg, zg)[3] <= 10 * U
