"""FP64 reference solutions and error measures for LSE and GLS.

TEST INFRASTRUCTURE ONLY (see the package docstring): the product path never
imports this module.

Everything here is a plain transcription of the definitions in the paper,
computed in float64 with numpy / scipy (LAPACK) routines as the building
blocks; no blocking, fusion or reordering beyond what the definitions state.

Notation follows the paper: LSE uses A (m x n), B (p x n), b, d; GLS uses
W (n x m), V (n x p), d.  The LSE iterate of the 3-block augmented system is
[r; -v; x] and the GLS iterate is [y; -z; x].
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
from scipy.sparse.linalg import LinearOperator, onenormest

__all__ = [
    "grq", "lse_solve", "gqr", "gls_solve",
    "lse_augmented", "gls_augmented",
    "lse_residual", "gls_residual", "lse_scales", "gls_scales",
    "lse_berr", "gls_berr",
    "lse_err1", "lse_err2", "gls_err1", "gls_err2",
    "skeel_cond_block", "lse_cond_x", "gls_cond_xy",
    "skeel_cond_block_est", "lse_cond_x_est", "gls_cond_xy_est",
    "check_lse_assumptions", "check_gls_assumptions",
]

_nrm = np.linalg.norm


def _fro(M):
    return float(np.linalg.norm(M, "fro")) if M.size else 0.0


def _utri_solve(T, rhs, trans=False):
    if T.shape[0] == 0:
        return np.zeros(0)
    return sla.solve_triangular(T, rhs, lower=False, trans="T" if trans else "N")


# --------------------------------------------------------------------------
# Assumptions (eq. assump:lse, eq. assump:gls)
# --------------------------------------------------------------------------

def check_lse_assumptions(A, B, rtol=None):
    """rank(B) = p and rank([A; B]) = n with p <= n <= m + p (Section 1)."""
    m, n = A.shape
    p = B.shape[0]
    if not (p <= n <= m + p):
        return False
    rb = np.linalg.matrix_rank(B, tol=rtol) if p else 0
    rab = np.linalg.matrix_rank(np.vstack([A, B]), tol=rtol)
    return rb == p and rab == n


def check_gls_assumptions(W, V, rtol=None):
    """rank([W, V]) = n and rank(W) = m with m <= n <= m + p (Section 1)."""
    n, m = W.shape
    p = V.shape[1]
    if not (m <= n <= m + p):
        return False
    return (np.linalg.matrix_rank(np.hstack([W, V]), tol=rtol) == n
            and np.linalg.matrix_rank(W, tol=rtol) == m)


# --------------------------------------------------------------------------
# LSE: null-space method via the GRQ factorization (Section 2.1)
# --------------------------------------------------------------------------

def grq(B, A):
    """GRQ factorization of (B, A): B = [0, R] Q and A = Z T Q.

    First an RQ factorization of B, then a QR factorization of A Q^T, as in
    Section 4.2 (the order LAPACK's xGGRQF uses).  Returns R (p x p upper
    triangular), T (m x n upper trapezoidal), Z (m x m) and Q (n x n), with Z
    and Q orthogonal and formed explicitly.
    """
    m, n = A.shape
    p = B.shape[0]
    if p > 0:
        Rf, Q = sla.rq(B, mode="full")          # B = Rf Q, Rf = [0, R]
        R = Rf[:, n - p:]
    else:
        R, Q = np.zeros((0, 0)), np.eye(n)
    Z, T = np.linalg.qr(A @ Q.T, mode="complete")
    return R, T, Z, Q


def lse_solve(A, B, b, d):
    """Solve min ||Ax - b|| s.t. Bx = d by the null-space method (Section 2.1).

    Steps: B = [0, R] Q, A = Z T Q; R y2 = d; c = Z^T b;
    T11 y1 = c1 - T12 y2; x = Q^T [y1; y2].  The auxiliary unknowns of the
    3-block system (eq. aug-LSE) are r = b - A x and v from
    R^T v = (Q A^T r)(n-p+1:n), the relation used for the initial v0 of
    Algorithm 2.  Returns (x, r, v).
    """
    A = np.asarray(A, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    d = np.asarray(d, dtype=np.float64)
    m, n = A.shape
    p = B.shape[0]
    R, T, Z, Q = grq(B, A)
    y2 = _utri_solve(R, d)
    c = Z.T @ b
    k = n - p
    T11 = T[:k, :k]
    T12 = T[:k, k:]
    y1 = _utri_solve(T11, c[:k] - T12 @ y2)
    x = Q.T @ np.concatenate([y1, y2])
    r = b - A @ x
    v = _utri_solve(R, (Q @ (A.T @ r))[k:], trans=True)
    return x, r, v


# --------------------------------------------------------------------------
# GLS: Paige's method via the GQR factorization (Section 2.2)
# --------------------------------------------------------------------------

def gqr(W, V):
    """GQR factorization of (W, V): W = Q [R; 0] and V = Q T Z.

    A QR factorization of W followed by an RQ factorization of Q^T V.
    Returns R (m x m upper triangular), T (n x p), Q (n x n), Z (p x p).
    """
    n, m = W.shape
    p = V.shape[1]
    Q, Rf = np.linalg.qr(W, mode="complete")
    R = Rf[:m, :m]
    T, Z = sla.rq(Q.T @ V, mode="full")         # Q^T V = T Z
    return R, T, Q, Z


def gls_solve(W, V, d):
    """Solve min ||y|| s.t. Wx + Vy = d by Paige's method (Section 2.2).

    Steps: W = Q [R; 0], V = Q T Z; c = Q^T d; T22 s2 = c2;
    R x = c1 - T12 s2; y = Z^T [0; s2].  The auxiliary unknown z of the
    3-block system (eq. aug-GLS) is z = Q [0; v] with T22^T v = (Z y)(p-n+m+1:p)
    (the initial z0 of Algorithm 4, read with Q rather than Q^H: rows one and
    three of eq. aug-GLS require W^T z = 0 and V^T z = y, which Q [0; v]
    satisfies and Q^T [0; v] does not).  Returns (x, y, z).
    """
    W = np.asarray(W, dtype=np.float64)
    V = np.asarray(V, dtype=np.float64)
    d = np.asarray(d, dtype=np.float64)
    n, m = W.shape
    p = V.shape[1]
    R, T, Q, Z = gqr(W, V)
    k = n - m                       # size of T22
    j = p - k                       # = p - n + m, width of T11
    c = Q.T @ d
    T22 = T[m:, j:]
    T12 = T[:m, j:]
    s2 = _utri_solve(T22, c[m:])
    x = _utri_solve(R, c[:m] - T12 @ s2)
    y = Z.T @ np.concatenate([np.zeros(j), s2])
    v = _utri_solve(T22, (Z @ y)[j:], trans=True)
    z = Q @ np.concatenate([np.zeros(m), v])
    return x, y, z


# --------------------------------------------------------------------------
# Augmented systems and their residuals (eqs. aug-LSE, aug-GLS)
# --------------------------------------------------------------------------

def lse_augmented(A, B):
    """[[I_m, 0, A], [0, 0, B], [A^T, B^T, 0]] acting on [r; -v; x]."""
    m, n = A.shape
    p = B.shape[0]
    N = m + p + n
    F = np.zeros((N, N))
    F[:m, :m] = np.eye(m)
    F[:m, m + p:] = A
    F[m:m + p, m + p:] = B
    F[m + p:, :m] = A.T
    F[m + p:, m:m + p] = B.T
    return F


def gls_augmented(W, V):
    """[[I_p, V^T, 0], [V, 0, W], [0, W^T, 0]] acting on [y; -z; x]."""
    n, m = W.shape
    p = V.shape[1]
    N = p + n + m
    F = np.zeros((N, N))
    F[:p, :p] = np.eye(p)
    F[:p, p:p + n] = V.T
    F[p:p + n, :p] = V
    F[p:p + n, p + n:] = W
    F[p + n:, p:p + n] = W.T
    return F


def lse_residual(A, B, b, d, x, r, v):
    """f1 = b - r - Ax, f2 = d - Bx, f3 = -A^T r + B^T v (Algorithm 2, refinement step)."""
    f1 = b - r - A @ x
    f2 = d - B @ x
    f3 = -(A.T @ r) + B.T @ v
    return f1, f2, f3


def gls_residual(W, V, d, x, y, z):
    """f1 = -y + V^T z, f2 = d - Wx - Vy, f3 = W^T z (Algorithm 4, refinement step)."""
    f1 = -y + V.T @ z
    f2 = d - W @ x - V @ y
    f3 = W.T @ z
    return f1, f2, f3


def lse_scales(A, B, b, d, x, r, v):
    """Right-hand sides of eq. lse-stop without the factor tol."""
    nA, nB = _fro(A), _fro(B)
    return (_nrm(b) + _nrm(r) + nA * _nrm(x),
            _nrm(d) + nB * _nrm(x),
            nA * _nrm(r) + nB * _nrm(v))


def gls_scales(W, V, d, x, y, z):
    """Right-hand sides of eq. gls-stop without the factor tol."""
    nW, nV = _fro(W), _fro(V)
    return (_nrm(y) + nV * _nrm(z),
            _nrm(d) + nW * _nrm(x) + nV * _nrm(y),
            nW * _nrm(z))


def _ratio(f, s):
    nf = float(_nrm(f))
    if nf == 0.0:
        return 0.0
    return nf / s if s > 0 else float("inf")


def lse_berr(A, B, b, d, x, r, v):
    """Blockwise normwise backward error: ||f_i|| / (scale_i of eq. lse-stop).

    The stopping test of eq. lse-stop holds with threshold tol exactly when
    every entry is <= tol.  Returns (berr1, berr2, berr3, max).
    """
    f = lse_residual(A, B, b, d, x, r, v)
    s = lse_scales(A, B, b, d, x, r, v)
    e = [_ratio(fi, si) for fi, si in zip(f, s)]
    return e[0], e[1], e[2], max(e)


def gls_berr(W, V, d, x, y, z):
    """Blockwise normwise backward error for eq. gls-stop.  Returns (e1, e2, e3, max)."""
    f = gls_residual(W, V, d, x, y, z)
    s = gls_scales(W, V, d, x, y, z)
    e = [_ratio(fi, si) for fi, si in zip(f, s)]
    return e[0], e[1], e[2], max(e)


# --------------------------------------------------------------------------
# Accuracy metrics of Tables 4 and 5
# --------------------------------------------------------------------------

def lse_err1(B, d, x):
    """err-1 of Table 4: ||Bx - d|| / (||B||_F ||x|| + ||d||)."""
    return float(_nrm(B @ x - d) / (_fro(B) * _nrm(x) + _nrm(d)))


def lse_err2(A, b, x, x_ref):
    """err-2 of Table 4: | ||Ax - b|| / ||A x_ref - b|| - 1 |."""
    return float(abs(_nrm(A @ x - b) / _nrm(A @ x_ref - b) - 1.0))


def gls_err1(W, V, d, x, y):
    """err-1 of Table 5: ||Wx + Vy - d|| / (||W||_F ||x|| + ||V||_F ||y|| + ||d||)."""
    return float(_nrm(W @ x + V @ y - d) / (_fro(W) * _nrm(x) + _fro(V) * _nrm(y) + _nrm(d)))


def gls_err2(y, y_ref):
    """err-2 of Table 5: | ||y|| / ||y_ref|| - 1 |."""
    return float(abs(_nrm(y) / _nrm(y_ref) - 1.0))


# --------------------------------------------------------------------------
# Componentwise (Skeel) condition number, restricted to one block
# --------------------------------------------------------------------------

def skeel_cond_block(F, u, sl):
    """|| (|F^-1| |F| |u|)[sl] ||_inf / || u[sl] ||_inf.

    The quantity cond(F~, u~) of Theorems 4.4 and 4.6, restricted to the rows
    of the block sl.  Computed with a dense inverse, so only for modest N.
    """
    Finv = np.linalg.inv(F)
    t = np.abs(Finv) @ (np.abs(F) @ np.abs(u))
    den = np.max(np.abs(u[sl]))
    return float(np.max(t[sl]) / den) if den > 0 else float("inf")


def lse_cond_x(A, B, x, r, v):
    """Skeel condition number of the x-block of eq. aug-LSE at [r; -v; x]."""
    m, n = A.shape
    p = B.shape[0]
    F = lse_augmented(A, B)
    u = np.concatenate([r, -v, x])
    return skeel_cond_block(F, u, slice(m + p, m + p + n))


def gls_cond_xy(W, V, x, y, z):
    """Skeel condition numbers of the x- and y-blocks of eq. aug-GLS at [y; -z; x]."""
    n, m = W.shape
    p = V.shape[1]
    F = gls_augmented(W, V)
    u = np.concatenate([y, -z, x])
    return (skeel_cond_block(F, u, slice(p + n, p + n + m)),
            skeel_cond_block(F, u, slice(0, p)))


def skeel_cond_block_est(F, u, sl):
    """Estimate of skeel_cond_block(F, u, sl) for large N, without F^-1.

    With g = |F| |u| (nonnegative), the block's entries of |F^-1| g are the
    column sums of |S| for S = diag(g) F^-T P, where P keeps the block's
    coordinates and zeroes the rest; so || (|F^-1| g)[sl] ||_inf = ||S||_1.
    The block 1-norm estimator of Higham and Tisseur
    (scipy.sparse.linalg.onenormest) estimates ||S||_1 from products with S
    and S^T, each one solve with an LU factorization of F.  The estimate is a
    lower bound of the exact value and equals it in most cases.
    """
    N = F.shape[0]
    lu = sla.lu_factor(F)
    g = np.abs(F) @ np.abs(u)
    keep = np.zeros(N)
    keep[sl] = 1.0

    def matvec(y):
        return g * sla.lu_solve(lu, keep * np.ravel(y), trans=1)

    def rmatvec(w):
        return keep * sla.lu_solve(lu, g * np.ravel(w))

    op = LinearOperator((N, N), matvec=matvec, rmatvec=rmatvec, dtype=np.float64)
    est = float(onenormest(op, t=2, itmax=6))
    den = np.max(np.abs(u[sl]))
    return est / den if den > 0 else float("inf")


def lse_cond_x_est(A, B, x, r, v):
    """lse_cond_x through skeel_cond_block_est (large systems)."""
    m, n = A.shape
    p = B.shape[0]
    u = np.concatenate([r, -v, x])
    return skeel_cond_block_est(lse_augmented(A, B), u, slice(m + p, m + p + n))


def gls_cond_xy_est(W, V, x, y, z):
    """gls_cond_xy through skeel_cond_block_est (large systems)."""
    n, m = W.shape
    p = V.shape[1]
    F = gls_augmented(W, V)
    u = np.concatenate([y, -z, x])
    return (skeel_cond_block_est(F, u, slice(p + n, p + n + m)),
            skeel_cond_block_est(F, u, slice(0, p)))
