"""CPU pins of the extended-precision references (oracle/extended.py): the
exact residual against hand-worked integer values, against mpmath at 60
digits and against the FP64 residual where FP64 is exact; the mpmath
solutions against the FP64 oracle on well-conditioned data and against the
closed form of a square constrained system."""
import mpmath
import numpy as np

from oracle import direct, extended

U = 2.0 ** -53


def test_exact_residual_hand_worked():
    # A = [[1, 2], [3, 4], [5, 6]], B = [[1, 1]], b = [1, 2, 3], d = [4]
    # at x = [1, -1], r = [0.5, 0, -0.5], v = [2]:
    # A x = [-1, -1, -1]; f1 = b - r - Ax = [1.5, 3, 4.5]
    # B x = 0; f2 = 4
    # A^T r = [0.5 - 2.5, 1 - 3] = [-2, -2]; B^T v = [2, 2]; f3 = [4, 4]
    A = np.array([[1.0, 2.0], [3.0, 4.0], [5.0, 6.0]])
    B = np.array([[1.0, 1.0]])
    f1, f2, f3 = extended.lse_residual_exact(A, B, np.array([1.0, 2.0, 3.0]), np.array([4.0]),
                                             np.array([1.0, -1.0]), np.array([0.5, 0.0, -0.5]),
                                             np.array([2.0]))
    assert list(f1) == [1.5, 3.0, 4.5] and list(f2) == [4.0] and list(f3) == [4.0, 4.0]
    # GLS: W = [[1], [2]], V = [[1, 0], [1, 1]], d = [3, 5] at x = [1], y = [1, 1], z = [1, -1]:
    # V^T z = [0, -1]; f1 = -y + V^T z = [-1, -2]; Wx + Vy = [2, 4]; f2 = [1, 1];
    # W^T z = -1; f3 = [-1]
    W = np.array([[1.0], [2.0]])
    V = np.array([[1.0, 0.0], [1.0, 1.0]])
    g1, g2, g3 = extended.gls_residual_exact(W, V, np.array([3.0, 5.0]), np.array([1.0]),
                                             np.array([1.0, 1.0]), np.array([1.0, -1.0]))
    assert list(g1) == [-1.0, -2.0] and list(g2) == [1.0, 1.0] and list(g3) == [-1.0]


def test_exact_residual_matches_mpmath_and_cancellation():
    rng = np.random.default_rng(31)
    m, n, p = 9, 5, 2
    A, B = rng.standard_normal((m, n)), rng.standard_normal((p, n))
    x, r, v = rng.standard_normal(n), rng.standard_normal(m), rng.standard_normal(p)
    # right-hand sides that nearly cancel: b = r + A x rounded, d = B x rounded
    b = r + A @ x
    d = B @ x
    f1, f2, f3 = extended.lse_residual_exact(A, B, b, d, x, r, v)
    with mpmath.workdps(60):
        for i in range(m):
            s = mpmath.mpf(float(b[i])) - mpmath.mpf(float(r[i])) - mpmath.fsum(
                mpmath.mpf(float(A[i, j])) * mpmath.mpf(float(x[j])) for j in range(n))
            assert f1[i] == float(s)
        for j in range(n):
            s = -mpmath.fsum(mpmath.mpf(float(A[i, j])) * mpmath.mpf(float(r[i])) for i in range(m)) \
                + mpmath.fsum(mpmath.mpf(float(B[i, j])) * mpmath.mpf(float(v[i])) for i in range(p))
            assert f3[j] == float(s)
    # the FP64 residual of this iterate is rounding noise of size u |terms|,
    # the exact one is the true (tiny) residual: they differ
    g1 = b - r - A @ x
    scale = np.abs(b) + np.abs(r) + np.abs(A) @ np.abs(x)
    assert np.all(np.abs(f1) <= 4 * U * scale)
    assert np.max(np.abs(g1 - f1)) <= 8 * n * U * np.max(scale)


def test_exact_residual_equals_fp64_when_fp64_is_exact():
    # small integers: every FP64 operation is exact, so both agree bit for bit
    rng = np.random.default_rng(32)
    W = rng.integers(-5, 6, (7, 3)).astype(float)
    V = rng.integers(-5, 6, (7, 6)).astype(float)
    d = rng.integers(-9, 10, 7).astype(float)
    x, y, z = (rng.integers(-3, 4, k).astype(float) for k in (3, 6, 7))
    f = extended.gls_residual_exact(W, V, d, x, y, z)
    g = direct.gls_residual(W, V, d, x, y, z)
    for a, c in zip(f, g):
        assert np.array_equal(a, c)


def test_mp_solutions_against_fp64_oracle():
    rng = np.random.default_rng(33)
    A, B = rng.standard_normal((12, 6)), rng.standard_normal((2, 6))
    b, d = rng.standard_normal(12), rng.standard_normal(2)
    x, r, v = extended.lse_solve_mp(A, B, b, d, dps=40)
    xo, ro, vo = direct.lse_solve(A, B, b, d)
    assert np.max(np.abs(x - xo)) <= 1e-13 * np.max(np.abs(xo))
    assert np.max(np.abs(v - vo)) <= 1e-12 * np.max(np.abs(vo))
    W, V, dd = rng.standard_normal((8, 3)), rng.standard_normal((8, 6)), rng.standard_normal(8)
    xg, yg, zg = extended.gls_solve_mp(W, V, dd, dps=40)
    xr, yr, zr = direct.gls_solve(W, V, dd)
    assert np.max(np.abs(xg - xr)) <= 1e-13 * np.max(np.abs(xr))
    assert np.max(np.abs(yg - yr)) <= 1e-13 * np.max(np.abs(yr))


def test_mp_lse_square_stack_closed_form():
    # n = m + p: [A; B] is square and x = [A; B]^{-1} [b; d] exactly, r = 0
    rng = np.random.default_rng(34)
    A, B = rng.standard_normal((4, 6)), rng.standard_normal((2, 6))
    b, d = rng.standard_normal(4), rng.standard_normal(2)
    x, r, _ = extended.lse_solve_mp(A, B, b, d, dps=40)
    with mpmath.workdps(40):
        S = mpmath.matrix(np.vstack([A, B]).tolist())
        ref = mpmath.lu_solve(S, mpmath.matrix(np.concatenate([b, d]).tolist()))
        assert max(abs(float(ref[i]) - x[i]) for i in range(6)) <= 2 * U * max(abs(float(t)) for t in ref)
    assert np.max(np.abs(r)) <= 1e-30
