"""CPU checks of the seeded input generators (paper_2406_16499_amd/workloads.py):
the conditioning they promise, orthogonality of the Haar factors, the shape
rules of the batch recipe, and reproducibility from the seed."""
import math
import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from paper_2406_16499_amd import workloads as wl  # noqa: E402


def test_haar_columns_are_orthonormal():
    Q = wl.haar(np.random.default_rng(1), 50, 20)
    assert np.max(np.abs(Q.T @ Q - np.eye(20))) < 1e-13


@pytest.mark.parametrize("rows,cols,kappa", [(40, 25, 1e3), (25, 40, 1e7), (30, 30, 10.0)])
def test_conditioned_has_the_prescribed_spectrum(rows, cols, kappa):
    M = wl.conditioned(np.random.default_rng(2), rows, cols, kappa)
    s = np.linalg.svd(M, compute_uv=False)
    assert s[0] == pytest.approx(1.0, rel=1e-12)
    assert s[0] / s[-1] == pytest.approx(kappa, rel=1e-6)
    k = min(rows, cols)
    assert np.allclose(s, wl.log_spaced(k, kappa), rtol=1e-9)


def test_paper_pairs_condition_the_stacked_matrix():
    P = wl.lse_paper_pair(np.random.default_rng(3), 60, 20, 5, 1e5)
    assert np.linalg.cond(np.vstack([P.A, P.B])) == pytest.approx(1e5, rel=1e-6)
    G = wl.gls_paper_pair(np.random.default_rng(4), 20, 6, 40, 1e4)
    assert np.linalg.cond(np.hstack([G.W, G.V])) == pytest.approx(1e4, rel=1e-6)


def test_batch_recipe_shapes_and_reproducibility():
    probs = list(wl.batch_instances(seed=9, count=60, kappa_max=1e6, m_range=(64, 200)))
    kinds = set()
    for P in probs:
        if hasattr(P, "b"):
            m, n, p = P.shape
            kinds.add("lse")
            assert 64 <= m <= 200 and 32 <= n <= max(32, m // 2) and 4 <= p <= max(4, n // 4)
            assert p <= n <= m + p
        else:
            n, m, p = P.shape
            kinds.add("gls")
            assert 64 <= p <= 200 and 32 <= n <= max(32, p // 2) and 4 <= m <= max(4, n // 4)
            assert m <= n <= m + p
    assert kinds == {"lse", "gls"}
    # instance i is regenerated from its own spawned seed, alone
    again = list(wl.batch_instances(seed=9, count=60, kappa_max=1e6, m_range=(64, 200)))
    for P, Q in zip(probs, again):
        a = P.A if hasattr(P, "b") else P.W
        b = Q.A if hasattr(Q, "b") else Q.W
        assert np.array_equal(a, b)


def test_log_spaced_endpoints():
    s = wl.log_spaced(7, 1e6)
    assert s[0] == 1.0 and s[-1] == pytest.approx(1e-6, rel=1e-12)
    assert np.allclose(np.diff(np.log10(s)), -1.0)
