"""The mixed-precision refinement method on the CPU (the paper's algorithms).

TEST INFRASTRUCTURE ONLY (see the package docstring).

This module follows the paper's steps in its order and notation:

* Algorithm 1 (correction solver, LSE) and Algorithm 3 (correction solver,
  GLS), the latter with the readings below;
* Algorithm 2 (MPLSE) and Algorithm 4 (MPGLS): factorization at precision
  u_f, initial guess, then classical refinement with residuals in FP64 until
  the stopping tests eq. lse-stop / eq. gls-stop hold;
* GMRES-based refinement (Section 5) with the block-diagonal split
  preconditioners eq. lse-bdpre-mlarge (LSE, m >= n), eq. lse-bdpre-nlarge
  (LSE, n > m), eq. gls-bdpre-plarge (GLS, n <= p) and eq. gls-bdpre-nlarge
  (GLS, n > p) on the scaled systems of eq. lse-limit-notation and
  eq. gls-limit-notation.  GMRES runs in FP64 (Section 6.1).

The low-precision factorization uses LAPACK in the precision of `uf`
(numpy / scipy call sgeqrf / sgerqf for float32 inputs), and the factors are
formed explicitly.  Only float32 and float64 are supported as u_f here.

Readings of the paper used in this module:
* Algorithm 3 solves T22 g2 = u2 for g2 (as eq. gls-solver derives), not the
  transposed system printed in the algorithm.
* The correction of z is dz = -Q h: with h defined as in the text the three
  equations of eq. gls-solver hold for h = -Q^T dz, and the ENSURE clause of
  Algorithm 3 holds for x2 = -Q h.
* z0 = Q [0; v] (Algorithm 4's initial z, read with Q instead of Q^H).
* The default tolerance is 1e-14 and residuals are always formed in FP64.
* When the initial r (LSE) or y (GLS) is zero, alpha falls back to
  2^(-1/2) min |diag| of the triangle of the second factorization (T1 for
  LSE, T2 for GLS), an estimate of the smallest singular value that keeps
  the scaled system well defined.
"""
from __future__ import annotations

import dataclasses
from typing import Callable, List, Optional

import numpy as np
import scipy.linalg as sla

from . import direct

__all__ = [
    "grq_factors", "gqr_factors", "correction_lse", "correction_gls",
    "lse_bd_triangles", "gls_bd_triangles",
    "mplse", "mpgls", "bd_operators_lse", "bd_operators_gls", "gmres",
    "mplse_gmres_bd", "mpgls_gmres_bd", "IRResult",
]


@dataclasses.dataclass
class IRResult:
    x: np.ndarray
    aux1: np.ndarray          # r (LSE) or y (GLS)
    aux2: np.ndarray          # v (LSE) or z (GLS)
    converged: bool
    steps: int                # number of corrections applied
    inner: int                # total GMRES iterations (0 for classical IR)
    berr_history: List[float]


def _ut(T, rhs, trans=False):
    if T.shape[0] == 0:
        return np.zeros(0, dtype=rhs.dtype)
    return sla.solve_triangular(T, rhs, lower=False, trans="T" if trans else "N",
                                check_finite=False)


# --------------------------------------------------------------------------
# Low-precision generalized factorizations (Section 4.2)
# --------------------------------------------------------------------------

def grq_factors(B, A, uf=np.float32):
    """GRQ of (B, A) at precision uf: B = [0, R] Q, A Q^T = Z T (explicit Q, Z)."""
    m, n = A.shape
    p = B.shape[0]
    Bf = np.asarray(B, dtype=uf)
    Af = np.asarray(A, dtype=uf)
    if p > 0:
        Rf, Q = sla.rq(Bf, mode="full")
        R = Rf[:, n - p:]
    else:
        R, Q = np.zeros((0, 0), dtype=uf), np.eye(n, dtype=uf)
    Z, T = np.linalg.qr(Af @ Q.T, mode="complete")
    return R, T, Z, Q


def gqr_factors(W, V, uf=np.float32):
    """GQR of (W, V) at precision uf: W = Q [R; 0], Q^T V = T Z."""
    n, m = W.shape
    Wf = np.asarray(W, dtype=uf)
    Vf = np.asarray(V, dtype=uf)
    Q, Rf = np.linalg.qr(Wf, mode="complete")
    R = Rf[:m, :m]
    T, Z = sla.rq(Q.T @ Vf, mode="full")
    return R, T, Q, Z


# --------------------------------------------------------------------------
# Correction solvers
# --------------------------------------------------------------------------

def correction_lse(R, T, Z, Q, f1, f2, f3, us=np.float32):
    """Algorithm 1 at precision us.  Returns (dr, dv, dx) in float64 with
    [[I,0,A],[0,0,B],[A^T,B^T,0]] [dr; -dv; dx] = [f1; f2; f3]."""
    p = R.shape[0]
    n = Q.shape[0]
    k = n - p
    R, T, Z, Q = (np.asarray(M, dtype=us) for M in (R, T, Z, Q))
    f1, f2, f3 = (np.asarray(f, dtype=us) for f in (f1, f2, f3))
    T11, T12, T22 = T[:k, :k], T[:k, k:], T[k:, k:]
    u = Q @ f3
    w = Z.T @ f1
    u1, u2 = u[:k], u[k:]
    w1, w2 = w[:k], w[k:]
    y2 = _ut(R, f2)
    q1 = _ut(T11, u1, trans=True)
    y1 = _ut(T11, w1 - q1 - T12 @ y2)
    q2 = w2 - T22 @ y2
    x1 = Z @ np.concatenate([q1, q2])
    x3 = Q.T @ np.concatenate([y1, y2])
    x2 = _ut(R, T12.T @ q1 + T22.T @ q2 - u2, trans=True)
    return (x1.astype(np.float64), x2.astype(np.float64), x3.astype(np.float64))


def correction_gls(R, T, Q, Z, f1, f2, f3, us=np.float32):
    """Algorithm 3 at precision us (with the readings in the module docstring).

    Returns (dy, dz, dx) in float64 with
    [[I,V^T,0],[V,0,W],[0,W^T,0]] [dy; -dz; dx] = [f1; f2; f3].
    """
    m = R.shape[0]
    n = Q.shape[0]
    p = Z.shape[0]
    k = n - m
    j = p - k
    R, T, Q, Z = (np.asarray(M, dtype=us) for M in (R, T, Q, Z))
    f1, f2, f3 = (np.asarray(f, dtype=us) for f in (f1, f2, f3))
    T11, T12, T22 = T[:m, :j], T[:m, j:], T[m:, j:]
    u = Q.T @ f2
    w = Z @ f1
    u1, u2 = u[:m], u[m:]
    w1, w2 = w[:j], w[j:]
    h1 = _ut(R, f3, trans=True)
    g2 = _ut(T22, u2)                            # T22 g2 = u2
    h2 = _ut(T22, w2 - g2 - T12.T @ h1, trans=True)
    g1 = w1 - T11.T @ h1
    dy = Z.T @ np.concatenate([g1, g2])
    dz = -(Q @ np.concatenate([h1, h2]))         #   (dz = -Q h)
    dx = _ut(R, u1 - T11 @ g1 - T12 @ g2)
    return (dy.astype(np.float64), dz.astype(np.float64), dx.astype(np.float64))


# --------------------------------------------------------------------------
# Initial guesses at u_f (Algorithms 2 and 4)
# --------------------------------------------------------------------------

def _lse_initial(A, B, b, d, R, T, Z, Q, uf):
    m, n = A.shape
    p = B.shape[0]
    k = n - p
    bf, df = b.astype(uf), d.astype(uf)
    y2 = _ut(R, df)
    c = Z.T @ bf
    y1 = _ut(T[:k, :k], c[:k] - T[:k, k:] @ y2)
    x0 = (Q.T @ np.concatenate([y1, y2])).astype(np.float64)
    r0 = (bf - A.astype(uf) @ x0.astype(uf)).astype(np.float64)   # at u_f
    Atr = A.T @ r0                                                  # A^T r at u_r
    v0 = _ut(R, (Q @ Atr.astype(uf))[k:], trans=True).astype(np.float64)
    return x0, r0, v0


def _gls_initial(W, V, d, R, T, Q, Z, uf):
    n, m = W.shape
    p = V.shape[1]
    k = n - m
    j = p - k
    c = Q.T @ d.astype(uf)
    s2 = _ut(T[m:, j:], c[m:])
    x0 = _ut(R, c[:m] - T[:m, j:] @ s2).astype(np.float64)
    y0 = (Z.T @ np.concatenate([np.zeros(j, dtype=uf), s2])).astype(np.float64)
    vv = _ut(T[m:, j:], (Z @ y0.astype(uf))[j:], trans=True)
    z0 = (Q @ np.concatenate([np.zeros(m, dtype=uf), vv])).astype(np.float64)
    return x0, y0, z0


def _stop(f, s, tol):
    return all(np.linalg.norm(fi) <= tol * si for fi, si in zip(f, s))


def _berr(f, s):
    out = 0.0
    for fi, si in zip(f, s):
        nf = float(np.linalg.norm(fi))
        if nf > 0.0:
            out = max(out, nf / si if si > 0 else float("inf"))
    return out


# --------------------------------------------------------------------------
# Algorithm 2 (MPLSE) and Algorithm 4 (MPGLS)
# --------------------------------------------------------------------------

def mplse(A, B, b, d, uf=np.float32, us=None, tol=1e-14, maxit=40):
    """Algorithm 2: mixed-precision classical refinement for LSE."""
    us = uf if us is None else us
    A, B, b, d = (np.asarray(a, dtype=np.float64) for a in (A, B, b, d))
    R, T, Z, Q = grq_factors(B, A, uf)
    x, r, v = _lse_initial(A, B, b, d, R, T, Z, Q, uf)
    hist = []
    for i in range(maxit + 1):
        f = direct.lse_residual(A, B, b, d, x, r, v)                # FP64 residual
        s = direct.lse_scales(A, B, b, d, x, r, v)
        hist.append(_berr(f, s))
        if not np.all([np.all(np.isfinite(fi)) for fi in f]):
            return IRResult(x, r, v, False, i, 0, hist)
        if _stop(f, s, tol):
            return IRResult(x, r, v, True, i, 0, hist)
        if i == maxit:
            break
        dr, dv, dx = correction_lse(R, T, Z, Q, *f, us=us)
        r, v, x = r + dr, v + dv, x + dx
    return IRResult(x, r, v, False, maxit, 0, hist)


def mpgls(W, V, d, uf=np.float32, us=None, tol=1e-14, maxit=40):
    """Algorithm 4: mixed-precision classical refinement for GLS."""
    us = uf if us is None else us
    W, V, d = (np.asarray(a, dtype=np.float64) for a in (W, V, d))
    R, T, Q, Z = gqr_factors(W, V, uf)
    x, y, z = _gls_initial(W, V, d, R, T, Q, Z, uf)
    hist = []
    for i in range(maxit + 1):
        f = direct.gls_residual(W, V, d, x, y, z)                   # FP64 residual
        s = direct.gls_scales(W, V, d, x, y, z)
        hist.append(_berr(f, s))
        if not np.all([np.all(np.isfinite(fi)) for fi in f]):
            return IRResult(x, y, z, False, i, 0, hist)
        if _stop(f, s, tol):
            return IRResult(x, y, z, True, i, 0, hist)
        if i == maxit:
            break
        dy, dz, dx = correction_gls(R, T, Q, Z, *f, us=us)
        x, y, z = x + dx, y + dy, z + dz
    return IRResult(x, y, z, False, maxit, 0, hist)


# --------------------------------------------------------------------------
# GMRES (Saad-Schultz) in FP64 with classical Gram-Schmidt applied twice
# --------------------------------------------------------------------------

def gmres(apply: Callable[[np.ndarray], np.ndarray], rhs: np.ndarray,
          restart: int = 30, tol: float = 1e-10, maxit: int = 300):
    """Restarted GMRES from a zero initial guess.

    Stops when the Arnoldi residual estimate drops to tol * ||rhs|| or after
    maxit iterations in total.  Returns (solution, iterations, converged).
    """
    N = rhs.shape[0]
    x = np.zeros(N)
    beta0 = float(np.linalg.norm(rhs))
    if beta0 == 0.0:
        return x, 0, True
    its = 0
    r = rhs.copy()
    while its < maxit:
        beta = float(np.linalg.norm(r))
        if beta <= tol * beta0:
            return x, its, True
        kmax = min(restart, maxit - its)
        Vb = np.zeros((N, kmax + 1))
        H = np.zeros((kmax + 1, kmax))
        cs = np.zeros(kmax)
        sn = np.zeros(kmax)
        g = np.zeros(kmax + 1)
        g[0] = beta
        Vb[:, 0] = r / beta
        k_done = 0
        for k in range(kmax):
            w = apply(Vb[:, k])
            h = Vb[:, :k + 1].T @ w                 # classical Gram-Schmidt ...
            w = w - Vb[:, :k + 1] @ h
            h2 = Vb[:, :k + 1].T @ w                # ... applied twice
            w = w - Vb[:, :k + 1] @ h2
            h = h + h2
            hn = float(np.linalg.norm(w))
            H[:k + 1, k] = h
            H[k + 1, k] = hn
            if hn > 0:
                Vb[:, k + 1] = w / hn
            for i in range(k):                     # earlier Givens rotations
                t = cs[i] * H[i, k] + sn[i] * H[i + 1, k]
                H[i + 1, k] = -sn[i] * H[i, k] + cs[i] * H[i + 1, k]
                H[i, k] = t
            rho = np.hypot(H[k, k], H[k + 1, k])
            cs[k] = H[k, k] / rho if rho > 0 else 1.0
            sn[k] = H[k + 1, k] / rho if rho > 0 else 0.0
            H[k, k] = rho
            H[k + 1, k] = 0.0
            g[k + 1] = -sn[k] * g[k]
            g[k] = cs[k] * g[k]
            its += 1
            k_done = k + 1
            if abs(g[k + 1]) <= tol * beta0 or hn == 0.0:
                break
        yk = sla.solve_triangular(H[:k_done, :k_done], g[:k_done], lower=False)
        x = x + Vb[:, :k_done] @ yk
        r = rhs - apply(x)
        if abs(g[k_done]) <= tol * beta0:
            return x, its, True
    return x, its, bool(np.linalg.norm(r) <= tol * beta0)


# --------------------------------------------------------------------------
# Block-diagonal split preconditioners (Sections 5.2 and 5.3)
# --------------------------------------------------------------------------

def lse_bd_triangles(T, n, p):
    """U (n x n) and Y (p x p) of the LSE preconditioners, from T (m x n).

    m >= n (eq. lse-bdpre-mlarge): U = T1 = T(1:n, 1:n) and Y = S =
    T1(n-p+1:n, n-p+1:n).  n > m (eq. lse-bdpre-nlarge): T = [T1, T2] and
    U = [T1, T2; 0, I_(n-m)], Y = [T1(n-p+1:m, n-p+1:m), T2(n-p+1:m, :); 0, I_(n-m)],
    which is again the trailing p x p block of U.
    """
    T = np.asarray(T, np.float64)
    m = T.shape[0]
    U = np.zeros((n, n))
    t = min(m, n)
    U[:t, :] = T[:t, :n]
    for i in range(t, n):
        U[i, i] = 1.0
    return U, U[n - p:, n - p:]


def gls_bd_triangles(T, n, m):
    """U (n x n) and Y (m x m) of the GLS preconditioners, from T (n x p).

    n <= p (eq. gls-bdpre-plarge): T = [0, T2], U = T2 and Y = S = T2(1:m, 1:m).
    n > p (eq. gls-bdpre-nlarge): T = [T1; T2] and U = [I_(n-p), T1; 0, T2],
    Y = [I_(n-p), T1(:, 1:m-n+p); 0, T2(1:m-n+p, 1:m-n+p)], which is again the
    leading m x m block of U.
    """
    T = np.asarray(T, np.float64)
    p = T.shape[1]
    U = np.zeros((n, n))
    if n <= p:
        U[:, :] = T[:, p - n:]
    else:
        U[:, n - p:] = T
        for i in range(n - p):
            U[i, i] = 1.0
    return U, U[:m, :m]


def bd_operators_lse(A, B, R, T, Q, alpha, beta):
    """M_l, F~, M_r of eq. lse-bdpre-mlarge (m >= n) or eq. lse-bdpre-nlarge
    (n > m) as functions on R^(m+p+n).  Factors are promoted to FP64.
    """
    m, n = A.shape
    p = B.shape[0]
    R = np.asarray(R, np.float64)
    U, Y = lse_bd_triangles(T, n, p)
    Q = np.asarray(Q, np.float64)
    sa = np.sqrt(alpha)

    def Ml(u):
        a, b_, c = u[:m], u[m:m + p], u[m + p:]
        return np.concatenate([a / sa, Y @ _ut(R, b_) / (sa * beta),
                               sa * _ut(U, Q @ c, trans=True)])

    def Mr(u):
        a, b_, c = u[:m], u[m:m + p], u[m + p:]
        return np.concatenate([a / sa, _ut(R, Y.T @ b_, trans=True) / (sa * beta),
                               sa * (Q.T @ _ut(U, c))])

    def F(u):
        a, b_, c = u[:m], u[m:m + p], u[m + p:]
        return np.concatenate([alpha * a + A @ c, beta * (B @ c),
                               A.T @ a + beta * (B.T @ b_)])
    return Ml, F, Mr


def bd_operators_gls(W, V, R, T, Q, alpha, beta):
    """M_l, F~, M_r of eq. gls-bdpre-plarge (n <= p) or eq. gls-bdpre-nlarge
    (n > p) as functions on R^(p+n+m).  Factors are promoted to FP64.
    """
    n, m = W.shape
    p = V.shape[1]
    R = np.asarray(R, np.float64)
    U, Y = gls_bd_triangles(T, n, m)
    Q = np.asarray(Q, np.float64)
    sa = np.sqrt(alpha)

    def Ml(u):
        a, b_, c = u[:p], u[p:p + n], u[p + n:]
        return np.concatenate([a / sa, sa * _ut(U, Q.T @ b_),
                               Y.T @ _ut(R, c, trans=True) / (sa * beta)])

    def Mr(u):
        a, b_, c = u[:p], u[p:p + n], u[p + n:]
        return np.concatenate([a / sa, sa * (Q @ _ut(U, b_, trans=True)),
                               _ut(R, Y @ c) / (sa * beta)])

    def F(u):
        a, b_, c = u[:p], u[p:p + n], u[p + n:]
        return np.concatenate([alpha * a + V.T @ b_, V @ a + beta * (W @ c),
                               beta * (W.T @ b_)])
    return Ml, F, Mr


def mplse_gmres_bd(A, B, b, d, uf=np.float32, tol=1e-14, maxit=40, restart=30,
                   gmres_tol=1e-10, gmres_maxit=300, alpha=None, beta=1.0):
    """MPLSE-GMRES-BD: refinement with GMRES on the BD-preconditioned eq. lse-limit-notation."""
    A, B, b, d = (np.asarray(a, dtype=np.float64) for a in (A, B, b, d))
    m, n = A.shape
    p = B.shape[0]
    R, T, Z, Q = grq_factors(B, A, uf)
    x, r, v = _lse_initial(A, B, b, d, R, T, Z, Q, uf)
    if alpha is None:
        alpha = float(np.linalg.norm(r))
        if not alpha > 0:
            t = min(m, n)
            alpha = 2 ** -0.5 * float(np.min(np.abs(np.diag(np.asarray(T, np.float64)[:t, :t]))))
    Ml, F, Mr = bd_operators_lse(A, B, R, T, Q, alpha, beta)
    sa = np.sqrt(alpha)
    hist, inner = [], 0
    for i in range(maxit + 1):
        f = direct.lse_residual(A, B, b, d, x, r, v)
        s = direct.lse_scales(A, B, b, d, x, r, v)
        hist.append(_berr(f, s))
        if _stop(f, s, tol):
            return IRResult(x, r, v, True, i, inner, hist)
        if i == maxit or inner >= gmres_maxit:
            break
        st = np.concatenate([sa * f[0], sa * beta * f[1], f[2] / sa])
        w, its, _ = gmres(lambda u: Ml(F(Mr(u))), Ml(st), restart, gmres_tol,
                          gmres_maxit - inner)
        inner += its
        du = Mr(w)
        r = r + sa * du[:m]
        v = v - sa * beta * du[m:m + p]
        x = x + du[m + p:] / sa
    return IRResult(x, r, v, False, i, inner, hist)


def mpgls_gmres_bd(W, V, d, uf=np.float32, tol=1e-14, maxit=40, restart=30,
                   gmres_tol=1e-10, gmres_maxit=300, alpha=None, beta=1.0):
    """MPGLS-GMRES-BD: refinement with GMRES on the BD-preconditioned eq. gls-limit-notation."""
    W, V, d = (np.asarray(a, dtype=np.float64) for a in (W, V, d))
    n, m = W.shape
    p = V.shape[1]
    R, T, Q, Z = gqr_factors(W, V, uf)
    x, y, z = _gls_initial(W, V, d, R, T, Q, Z, uf)
    if alpha is None:
        alpha = float(np.linalg.norm(y))
        if not alpha > 0:
            T2 = np.asarray(T, np.float64)
            T2 = T2[:, p - n:] if n <= p else T2[n - p:, :]
            alpha = 2 ** -0.5 * float(np.min(np.abs(np.diag(T2))))
    Ml, F, Mr = bd_operators_gls(W, V, R, T, Q, alpha, beta)
    sa = np.sqrt(alpha)
    hist, inner = [], 0
    for i in range(maxit + 1):
        f = direct.gls_residual(W, V, d, x, y, z)
        s = direct.gls_scales(W, V, d, x, y, z)
        hist.append(_berr(f, s))
        if _stop(f, s, tol):
            return IRResult(x, y, z, True, i, inner, hist)
        if i == maxit or inner >= gmres_maxit:
            break
        st = np.concatenate([sa * f[0], f[1] / sa, sa * beta * f[2]])
        w, its, _ = gmres(lambda u: Ml(F(Mr(u))), Ml(st), restart, gmres_tol,
                          gmres_maxit - inner)
        inner += its
        du = Mr(w)
        y = y + sa * du[:p]
        z = z - du[p:p + n] / sa
        x = x + sa * beta * du[p + n:]
    return IRResult(x, y, z, False, i, inner, hist)
