"""FP64 reference solutions and error measures for complex LSE and GLS.

TEST INFRASTRUCTURE ONLY (see the package docstring): the product path never
imports this module.

The problems of Section 1 are stated over the complex field, with Hermitian
transposes.  This module is their plain transcription in complex128 with
numpy / scipy (LAPACK's complex routines) as the building blocks:

* LSE, min ||Ax - b||_2 s.t. Bx = d (A m x n, B p x n): the null-space
  method through the generalized RQ factorization B = [0, R] Q, A = Z T Q
  with unitary Q, Z (Section 2.1, with ^H in place of ^T);
* GLS, min ||y||_2 s.t. d = Wx + Vy (W n x m, V n x p): Paige's method
  through the generalized QR factorization W = Q [R; 0], V = Q T Z
  (Section 2.2);
* the 3-block augmented systems (eq. aug-LSE, eq. aug-GLS) with A^H, B^H,
  their residual blocks, the stop-test scales of eq. lse-stop / eq. gls-stop
  (Frobenius norms of the complex matrices), the blockwise backward errors,
  the err-1 / err-2 measures of Tables 4 and 5 and the Skeel condition
  number of a block (componentwise moduli).

Nothing here uses a real embedding of the complex data, so a GPU solve that
goes through one is checked against an independent computation.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

__all__ = [
    "zgrq", "zlse_solve", "zgqr", "zgls_solve",
    "zlse_augmented", "zgls_augmented", "zlse_residual", "zgls_residual",
    "zlse_scales", "zgls_scales", "zlse_berr", "zgls_berr",
    "zlse_err1", "zlse_err2", "zgls_err1", "zgls_err2",
    "zskeel_cond_block", "zlse_cond_x", "zgls_cond_xy",
]

_nrm = np.linalg.norm


def _c(a):
    return np.asarray(a, dtype=np.complex128)


def _fro(M):
    return float(np.linalg.norm(M, "fro")) if M.size else 0.0


def _H(M):
    return M.conj().T


def _utri_solve(T, rhs, herm=False):
    if T.shape[0] == 0:
        return np.zeros(0, dtype=np.complex128)
    return sla.solve_triangular(T, rhs, lower=False, trans="C" if herm else "N")


# --------------------------------------------------------------------------
# LSE over C (Section 2.1)
# --------------------------------------------------------------------------

def zgrq(B, A):
    """B = [0, R] Q and A = Z T Q with Q (n x n), Z (m x m) unitary: an RQ
    factorization of B, then a QR factorization of A Q^H.  Returns R, T, Z, Q."""
    m, n = A.shape
    p = B.shape[0]
    if p > 0:
        Rf, Q = sla.rq(B, mode="full")
        R = Rf[:, n - p:]
    else:
        R, Q = np.zeros((0, 0), dtype=np.complex128), np.eye(n, dtype=np.complex128)
    Z, T = np.linalg.qr(A @ _H(Q), mode="complete")
    return R, T, Z, Q


def zlse_solve(A, B, b, d):
    """Null-space solution of the complex LSE.

    R y2 = d; c = Z^H b; T11 y1 = c1 - T12 y2; x = Q^H [y1; y2]; r = b - Ax;
    v from R^H v = (Q A^H r)(n-p+1:n) (the third block row of eq. aug-LSE,
    A^H r = B^H v).  Returns (x, r, v)."""
    A, B, b, d = _c(A), _c(B), _c(b), _c(d)
    m, n = A.shape
    p = B.shape[0]
    R, T, Z, Q = zgrq(B, A)
    k = n - p
    y2 = _utri_solve(R, d)
    c = _H(Z) @ b
    y1 = _utri_solve(T[:k, :k], c[:k] - T[:k, k:] @ y2)
    x = _H(Q) @ np.concatenate([y1, y2])
    r = b - A @ x
    v = _utri_solve(R, (Q @ (_H(A) @ r))[k:], herm=True)
    return x, r, v


# --------------------------------------------------------------------------
# GLS over C (Section 2.2)
# --------------------------------------------------------------------------

def zgqr(W, V):
    """W = Q [R; 0] and Q^H V = T Z with Q (n x n), Z (p x p) unitary.
    Returns R (m x m), T (n x p), Q, Z."""
    n, m = W.shape
    p = V.shape[1]
    Q, Rf = np.linalg.qr(W, mode="complete")
    R = Rf[:m, :m]
    if p > 0:
        T, Z = sla.rq(_H(Q) @ V, mode="full")
    else:
        T, Z = np.zeros((n, 0), dtype=np.complex128), np.zeros((0, 0), dtype=np.complex128)
    return R, T, Q, Z


def zgls_solve(W, V, d):
    """Paige's solution of the complex GLS.

    c = Q^H d; T22 s2 = c2; R x = c1 - T12 s2; y = Z^H [0; s2]; the
    auxiliary z = Q [0; v] with T22^H v = (Z y)(p-n+m+1:p) (rows one and
    three of eq. aug-GLS: y = V^H z, W^H z = 0).  Returns (x, y, z)."""
    W, V, d = _c(W), _c(V), _c(d)
    n, m = W.shape
    p = V.shape[1]
    R, T, Q, Z = zgqr(W, V)
    k = n - m
    j = p - k
    c = _H(Q) @ d
    T22 = T[m:, j:]
    s2 = _utri_solve(T22, c[m:])
    x = _utri_solve(R, c[:m] - T[:m, j:] @ s2)
    y = _H(Z) @ np.concatenate([np.zeros(j, dtype=np.complex128), s2])
    v = _utri_solve(T22, (Z @ y)[j:], herm=True)
    z = Q @ np.concatenate([np.zeros(m, dtype=np.complex128), v])
    return x, y, z


# --------------------------------------------------------------------------
# Augmented systems, residuals, stop-test scales, backward errors
# --------------------------------------------------------------------------

def zlse_augmented(A, B):
    """[[I, 0, A], [0, 0, B], [A^H, B^H, 0]] acting on [r; -v; x]."""
    A, B = _c(A), _c(B)
    m, n = A.shape
    p = B.shape[0]
    F = np.zeros((m + p + n, m + p + n), dtype=np.complex128)
    F[:m, :m] = np.eye(m)
    F[:m, m + p:] = A
    F[m:m + p, m + p:] = B
    F[m + p:, :m] = _H(A)
    F[m + p:, m:m + p] = _H(B)
    return F


def zgls_augmented(W, V):
    """[[I, V^H, 0], [V, 0, W], [0, W^H, 0]] acting on [y; -z; x]."""
    W, V = _c(W), _c(V)
    n, m = W.shape
    p = V.shape[1]
    F = np.zeros((p + n + m, p + n + m), dtype=np.complex128)
    F[:p, :p] = np.eye(p)
    F[:p, p:p + n] = _H(V)
    F[p:p + n, :p] = V
    F[p:p + n, p + n:] = W
    F[p + n:, p:p + n] = _H(W)
    return F


def zlse_residual(A, B, b, d, x, r, v):
    """f1 = b - r - Ax, f2 = d - Bx, f3 = -A^H r + B^H v."""
    A, B = _c(A), _c(B)
    return b - r - A @ x, d - B @ x, -(_H(A) @ r) + _H(B) @ v


def zgls_residual(W, V, d, x, y, z):
    """f1 = -y + V^H z, f2 = d - Wx - Vy, f3 = W^H z."""
    W, V = _c(W), _c(V)
    return -y + _H(V) @ z, d - W @ x - V @ y, _H(W) @ z


def zlse_scales(A, B, b, d, x, r, v):
    """Right-hand sides of eq. lse-stop without tol (Frobenius norms of the complex A, B)."""
    nA, nB = _fro(_c(A)), _fro(_c(B))
    return (_nrm(b) + _nrm(r) + nA * _nrm(x), _nrm(d) + nB * _nrm(x), nA * _nrm(r) + nB * _nrm(v))


def zgls_scales(W, V, d, x, y, z):
    """Right-hand sides of eq. gls-stop without tol."""
    nW, nV = _fro(_c(W)), _fro(_c(V))
    return (_nrm(y) + nV * _nrm(z), _nrm(d) + nW * _nrm(x) + nV * _nrm(y), nW * _nrm(z))


def _ratio(f, s):
    nf = float(_nrm(f))
    if nf == 0.0:
        return 0.0
    return nf / s if s > 0 else float("inf")


def zlse_berr(A, B, b, d, x, r, v):
    """(berr1, berr2, berr3, max) of eq. lse-stop at [r; -v; x]."""
    f = zlse_residual(A, B, b, d, x, r, v)
    s = zlse_scales(A, B, b, d, x, r, v)
    e = [_ratio(fi, si) for fi, si in zip(f, s)]
    return e[0], e[1], e[2], max(e)


def zgls_berr(W, V, d, x, y, z):
    """(berr1, berr2, berr3, max) of eq. gls-stop at [y; -z; x]."""
    f = zgls_residual(W, V, d, x, y, z)
    s = zgls_scales(W, V, d, x, y, z)
    e = [_ratio(fi, si) for fi, si in zip(f, s)]
    return e[0], e[1], e[2], max(e)


# --------------------------------------------------------------------------
# Accuracy metrics of Tables 4 and 5, Skeel condition numbers
# --------------------------------------------------------------------------

def zlse_err1(B, d, x):
    """||Bx - d|| / (||B||_F ||x|| + ||d||)."""
    B = _c(B)
    return float(_nrm(B @ x - d) / (_fro(B) * _nrm(x) + _nrm(d)))


def zlse_err2(A, b, x, x_ref):
    """| ||Ax - b|| / ||A x_ref - b|| - 1 |."""
    A = _c(A)
    return float(abs(_nrm(A @ x - b) / _nrm(A @ x_ref - b) - 1.0))


def zgls_err1(W, V, d, x, y):
    """||Wx + Vy - d|| / (||W||_F ||x|| + ||V||_F ||y|| + ||d||)."""
    W, V = _c(W), _c(V)
    return float(_nrm(W @ x + V @ y - d) / (_fro(W) * _nrm(x) + _fro(V) * _nrm(y) + _nrm(d)))


def zgls_err2(y, y_ref):
    """| ||y|| / ||y_ref|| - 1 |."""
    return float(abs(_nrm(y) / _nrm(y_ref) - 1.0))


def zskeel_cond_block(F, u, sl):
    """|| (|F^-1| |F| |u|)[sl] ||_inf / || u[sl] ||_inf with complex moduli
    (dense inverse: modest N only)."""
    Finv = np.linalg.inv(F)
    t = np.abs(Finv) @ (np.abs(F) @ np.abs(u))
    den = np.max(np.abs(u[sl]))
    return float(np.max(t[sl]) / den) if den > 0 else float("inf")


def zlse_cond_x(A, B, x, r, v):
    """Skeel condition number of the x-block of the complex eq. aug-LSE."""
    m, n = np.shape(A)
    p = np.shape(B)[0]
    u = np.concatenate([r, -v, x])
    return zskeel_cond_block(zlse_augmented(A, B), u, slice(m + p, m + p + n))


def zgls_cond_xy(W, V, x, y, z):
    """Skeel condition numbers of the x- and y-blocks of the complex eq. aug-GLS."""
    n, m = np.shape(W)
    p = np.shape(V)[1]
    F = zgls_augmented(W, V)
    u = np.concatenate([y, -z, x])
    return (zskeel_cond_block(F, u, slice(p + n, p + n + m)), zskeel_cond_block(F, u, slice(0, p)))
