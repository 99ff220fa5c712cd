"""Seeded synthetic inputs for LSE and GLS problems.

This module only *draws* inputs; it holds none of the method's arithmetic, so
both the CPU oracle and the GPU path can take their inputs from it.

Problem statements (Section 1): LSE is  min ||Ax - b||  s.t.  Bx = d  with
A (m x n), B (p x n), p <= n <= m + p.  GLS is  min ||y||  s.t.  Wx + Vy = d
with W (n x m), V (n x p), m <= n <= m + p.  The C-ABI writes the GLS pair as
(A, B) = (W, V).

Matrices with a prescribed condition number are built as U diag(s) V^T with
Haar-distributed orthogonal factors (QR of a Gaussian matrix with the sign of
diag(R) folded into Q, after Mezzadri 2007) and singular values s log-spaced
from 1 down to 1/kappa.  The paper builds its own test matrices the same way
from a prescribed spectrum (Section 6.2, [A^H, B^H] = W1 Sigma W2).

All arrays are float64, column-major (Fortran order) so that they can be
handed to the column-major C-ABI without a copy.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Iterator, List, Optional

import numpy as np

__all__ = [
    "LSEProblem", "GLSProblem", "haar", "conditioned", "gaussian",
    "lse_gaussian", "lse_conditioned", "gls_gaussian", "gls_conditioned",
    "config1", "config2", "config3", "batch_instances", "describe",
]


@dataclasses.dataclass
class LSEProblem:
    """min ||A x - b|| s.t. B x = d."""
    A: np.ndarray
    B: np.ndarray
    b: np.ndarray
    d: np.ndarray
    kind: str = "lse"
    kappa_A: Optional[float] = None
    kappa_B: Optional[float] = None

    @property
    def shape(self):
        m, n = self.A.shape
        return m, n, self.B.shape[0]


@dataclasses.dataclass
class GLSProblem:
    """min ||y|| s.t. W x + V y = d."""
    W: np.ndarray
    V: np.ndarray
    d: np.ndarray
    kind: str = "gls"
    kappa_W: Optional[float] = None
    kappa_V: Optional[float] = None

    @property
    def shape(self):
        n, m = self.W.shape
        return n, m, self.V.shape[1]


def _f(a: np.ndarray) -> np.ndarray:
    return np.asfortranarray(a, dtype=np.float64)


def gaussian(rng: np.random.Generator, rows: int, cols: int) -> np.ndarray:
    return _f(rng.standard_normal((rows, cols)))


def haar(rng: np.random.Generator, rows: int, cols: int) -> np.ndarray:
    """rows x cols matrix with Haar-distributed orthonormal columns (rows >= cols)."""
    assert rows >= cols
    g = rng.standard_normal((rows, cols))
    q, r = np.linalg.qr(g, mode="reduced")
    sgn = np.sign(np.diag(r))
    sgn[sgn == 0] = 1.0
    return q * sgn[None, :]


def log_spaced(k: int, kappa: float) -> np.ndarray:
    """s_i = kappa^(-(i-1)/(k-1)), i = 1..k (s_1 = 1, s_k = 1/kappa)."""
    if k == 1:
        return np.ones(1)
    return kappa ** (-np.arange(k) / (k - 1.0))


def conditioned(rng: np.random.Generator, rows: int, cols: int, kappa: float) -> np.ndarray:
    """U diag(s) V^T with Haar U, V and log-spaced s from 1 to 1/kappa."""
    k = min(rows, cols)
    s = log_spaced(k, kappa)
    u = haar(rng, rows, k)
    v = haar(rng, cols, k)
    return _f((u * s[None, :]) @ v.T)


def lse_gaussian(rng, m, n, p) -> LSEProblem:
    return LSEProblem(gaussian(rng, m, n), gaussian(rng, p, n),
                      rng.standard_normal(m), rng.standard_normal(p))


def lse_conditioned(rng, m, n, p, kappa_A, kappa_B=None) -> LSEProblem:
    A = conditioned(rng, m, n, kappa_A)
    B = conditioned(rng, p, n, kappa_B) if kappa_B is not None else gaussian(rng, p, n)
    return LSEProblem(A, B, rng.standard_normal(m), rng.standard_normal(p),
                      kappa_A=kappa_A, kappa_B=kappa_B)


def gls_gaussian(rng, n, m, p) -> GLSProblem:
    return GLSProblem(gaussian(rng, n, m), gaussian(rng, n, p), rng.standard_normal(n))


def gls_conditioned(rng, n, m, p, kappa_V, kappa_W=None) -> GLSProblem:
    W = conditioned(rng, n, m, kappa_W) if kappa_W is not None else gaussian(rng, n, m)
    V = conditioned(rng, n, p, kappa_V)
    return GLSProblem(W, V, rng.standard_normal(n), kappa_W=kappa_W, kappa_V=kappa_V)


def lse_paper_pair(rng, m, n, p, kappa) -> LSEProblem:
    """LSE whose stacked [A^T, B^T] (n x (m+p)) has condition number kappa.

    The construction of Section 6.2: [A^T, B^T] = W1 Sigma W2 with orthogonal
    W1, W2 from QR factorizations of random matrices and a prescribed
    spectrum (here geometric from 1 to 1/kappa).
    """
    C = conditioned(rng, n, m + p, kappa)
    return LSEProblem(_f(C[:, :m].T), _f(C[:, m:].T), rng.standard_normal(m),
                      rng.standard_normal(p), kappa_A=kappa)


def paper_bases(rng, n, N):
    """Orthogonal factors of the paper's generator (Section 6.2): U (n x n)
    and V (N x n, orthonormal columns), both Haar.  One pair serves every
    condition number of a shape: lse_paper_from_bases / gls_paper_from_bases
    put the spectrum between them."""
    return haar(rng, n, n), haar(rng, N, n)


def lse_paper_from_bases(rng, U, V, m, p, kappa) -> LSEProblem:
    """LSE with [A^T, B^T] = U diag(s) V^T (n x (m+p)), s log-spaced 1 .. 1/kappa;
    b, d ~ N(0, 1) drawn from rng."""
    n = U.shape[0]
    C = (U * log_spaced(n, kappa)) @ V.T
    return LSEProblem(_f(C[:, :m].T), _f(C[:, m:m + p].T), rng.standard_normal(m),
                      rng.standard_normal(p), kappa_A=kappa)


def gls_paper_from_bases(rng, U, V, m, p, kappa) -> GLSProblem:
    """GLS with [W, V] = U diag(s) V^T (n x (m+p)); d ~ N(0, 1) drawn from rng."""
    n = U.shape[0]
    C = (U * log_spaced(n, kappa)) @ V.T
    return GLSProblem(_f(C[:, :m]), _f(C[:, m:m + p]), rng.standard_normal(n), kappa_V=kappa)


def gls_paper_pair(rng, n, m, p, kappa) -> GLSProblem:
    """GLS whose [W, V] (n x (m+p)) has condition number kappa (Section 6.3)."""
    C = conditioned(rng, n, m + p, kappa)
    return GLSProblem(_f(C[:, :m]), _f(C[:, m:]), rng.standard_normal(n), kappa_V=kappa)


# --------------------------------------------------------------------------
# The named workloads (the benchmark configurations); smaller
# "scaled" variants keep the same structure for fast tests.
# --------------------------------------------------------------------------

def config1(seed: int = 1) -> LSEProblem:
    """Single real LSE, A 200x100, B 20x100, everything i.i.d. N(0,1)."""
    return lse_gaussian(np.random.default_rng(seed), 200, 100, 20)


def config2(seed: int = 2, m: int = 4096, n: int = 2048, p: int = 256,
            kappa: float = 1e4) -> LSEProblem:
    """Single large LSE: A = U diag(s) V^T (kappa(A)=1e4), B i.i.d. N(0,1)."""
    return lse_conditioned(np.random.default_rng(seed), m, n, p, kappa)


def config3(seed: int = 3, n: int = 4096, m: int = 1024, p: int = 4096,
            kappa: float = 1e6) -> GLSProblem:
    """Single GLS d = Wx + Vy: W i.i.d. N(0,1), V = U diag(s) V^T (kappa(V)=1e6)."""
    return gls_conditioned(np.random.default_rng(seed), n, m, p, kappa)


def batch_instances(seed: int = 4, count: int = 2000, kappa_max: float = 1e8,
                    m_range=(64, 1024), start: int = 0) -> Iterator[object]:
    """Mixed LSE/GLS instances of uneven size.

    LSE: m ~ U[m_lo, m_hi], n ~ U[32, m/2], p ~ U[4, n/4].
    GLS uses the mirrored shapes (p, n, m) of the LSE recipe, so that
    m <= n <= m + p holds: p ~ U[m_lo, m_hi], n ~ U[32, p/2], m ~ U[4, n/4].
    Both matrices of an instance are U diag(s) V^T with an independent
    kappa ~ log-uniform[1e1, kappa_max]; right-hand sides are N(0,1).
    Instance i draws from SeedSequence(seed).spawn(count)[i], so any
    instance can be regenerated on its own; `start` skips the first ones.
    """
    children = np.random.SeedSequence(seed).spawn(count)
    lo, hi = m_range
    for ss in children[start:]:
        rng = np.random.default_rng(ss)
        is_lse = rng.random() < 0.5
        big = int(rng.integers(lo, hi + 1))
        mid = int(rng.integers(32, max(32, big // 2) + 1))
        small = int(rng.integers(4, max(4, mid // 4) + 1))
        k1 = 10.0 ** rng.uniform(1.0, math.log10(kappa_max))
        k2 = 10.0 ** rng.uniform(1.0, math.log10(kappa_max))
        if is_lse:
            m, n, p = big, mid, small
            prob = LSEProblem(conditioned(rng, m, n, k1), conditioned(rng, p, n, k2),
                              rng.standard_normal(m), rng.standard_normal(p),
                              kappa_A=k1, kappa_B=k2)
        else:
            p, n, m = big, mid, small
            prob = GLSProblem(conditioned(rng, n, m, k1), conditioned(rng, n, p, k2),
                              rng.standard_normal(n), kappa_W=k1, kappa_V=k2)
        yield prob


def describe(prob) -> str:
    if prob.kind == "lse":
        m, n, p = prob.shape
        return f"LSE m={m} n={n} p={p}"
    n, m, p = prob.shape
    return f"GLS n={n} m={m} p={p}"
