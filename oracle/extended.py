"""Extended-precision references for the extra-precise residual (u_r = u^2).

TEST INFRASTRUCTURE ONLY (see the package docstring): the product path never
imports this module.

* lse_residual_exact / gls_residual_exact: the residual blocks of eq. aug-LSE
  / eq. aug-GLS at an FP64 iterate, computed exactly in rational arithmetic
  (every FP64 value is a rational number; fractions.Fraction adds and
  multiplies them without error) and rounded once to the nearest FP64
  number.  A double-double residual should agree with it to about one unit
  in the last place.
* lse_solve_mp / gls_solve_mp: the solution of the augmented system (the
  definition of the LSE / GLS solution, Section 2) in mpmath with `dps`
  decimal digits, rounded to FP64: the reference for forward errors at the
  level of u, which no FP64 solver reaches when the problem is ill
  conditioned.

Both are slow (pure Python); they serve small problems only.
"""
from __future__ import annotations

from fractions import Fraction

import mpmath
import numpy as np

__all__ = ["lse_residual_exact", "gls_residual_exact", "lse_solve_mp", "gls_solve_mp"]


def _fr(a):
    return [Fraction(float(t)) for t in np.ravel(a)]


def _matvec_exact(M, u):
    """Exact products M u for an FP64 matrix M (rows x cols) and vector u."""
    M = np.asarray(M, dtype=np.float64)
    rows, cols = M.shape
    uf = _fr(u)
    out = []
    for i in range(rows):
        s = Fraction(0)
        row = M[i]
        for j in range(cols):
            if row[j] != 0.0 and uf[j] != 0:
                s += Fraction(float(row[j])) * uf[j]
        out.append(s)
    return out


def lse_residual_exact(A, B, b, d, x, r, v):
    """f1 = b - r - Ax, f2 = d - Bx, f3 = -A^T r + B^T v, each entry exact, then
    rounded to FP64 once."""
    Ax = _matvec_exact(A, x)
    Bx = _matvec_exact(B, x)
    Atr = _matvec_exact(np.asarray(A).T, r)
    Btv = _matvec_exact(np.asarray(B).T, v)
    bf, rf, df = _fr(b), _fr(r), _fr(d)
    f1 = np.array([float(bf[i] - rf[i] - Ax[i]) for i in range(len(bf))])
    f2 = np.array([float(df[i] - Bx[i]) for i in range(len(df))])
    f3 = np.array([float(-Atr[i] + Btv[i]) for i in range(len(Atr))])
    return f1, f2, f3


def gls_residual_exact(W, V, d, x, y, z):
    """f1 = -y + V^T z, f2 = d - Wx - Vy, f3 = W^T z, exact then rounded once."""
    Vtz = _matvec_exact(np.asarray(V).T, z)
    Wx = _matvec_exact(W, x)
    Vy = _matvec_exact(V, y)
    Wtz = _matvec_exact(np.asarray(W).T, z)
    yf, df = _fr(y), _fr(d)
    f1 = np.array([float(-yf[i] + Vtz[i]) for i in range(len(yf))])
    f2 = np.array([float(df[i] - Wx[i] - Vy[i]) for i in range(len(df))])
    f3 = np.array([float(t) for t in Wtz])
    return f1, f2, f3


def _solve_mp(F, rhs, dps):
    with mpmath.workdps(dps):
        Fm = mpmath.matrix([[mpmath.mpf(float(t)) for t in row] for row in F])
        rm = mpmath.matrix([mpmath.mpf(float(t)) for t in rhs])
        sol = mpmath.lu_solve(Fm, rm)
        return np.array([float(sol[i]) for i in range(len(rhs))])


def lse_solve_mp(A, B, b, d, dps=50):
    """(x, r, v) of [[I, 0, A], [0, 0, B], [A^T, B^T, 0]] [r; -v; x] = [b; d; 0]
    solved with `dps` digits."""
    A, B = np.asarray(A, dtype=np.float64), np.asarray(B, dtype=np.float64)
    m, n = A.shape
    p = B.shape[0]
    N = m + p + n
    F = np.zeros((N, N))
    F[:m, :m] = np.eye(m)
    F[:m, m + p:] = A
    F[m:m + p, m + p:] = B
    F[m + p:, :m] = A.T
    F[m + p:, m:m + p] = B.T
    u = _solve_mp(F, np.concatenate([b, d, np.zeros(n)]), dps)
    return u[m + p:], u[:m], -u[m:m + p]


def gls_solve_mp(W, V, d, dps=50):
    """(x, y, z) of [[I, V^T, 0], [V, 0, W], [0, W^T, 0]] [y; -z; x] = [0; d; 0]
    solved with `dps` digits."""
    W, V = np.asarray(W, dtype=np.float64), np.asarray(V, dtype=np.float64)
    n, m = W.shape
    p = V.shape[1]
    N = p + n + m
    F = np.zeros((N, N))
    F[:p, :p] = np.eye(p)
    F[:p, p:p + n] = V.T
    F[p:p + n, :p] = V
    F[p:p + n, p + n:] = W
    F[p + n:, p:p + n] = W.T
    u = _solve_mp(F, np.concatenate([np.zeros(p), d, np.zeros(m)]), dps)
    return u[p + n:], u[:p], -u[p:p + n]
