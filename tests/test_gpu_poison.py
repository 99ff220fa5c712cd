"""The debug library liblsq_poison.so, whose kernels fill their LDS with NaN
bit patterns before first use (per instance in the persistent batch): every
path must still certify and match the oracle, which it cannot if any kernel
reads LDS that no thread of its work-group has written."""
import os
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
    if not os.path.exists(lsq.POISON_LIB_PATH):
        pytest.skip("liblsq_poison.so not built (python -m paper_2406_16499_amd.build poison)")
    hd = lsq.Handle(load_selector=False, lib=lsq.load_variant(lsq.POISON_LIB_PATH))
    yield hd
    hd.close()


def D(a):
    return lsq.colmajor(a)


def H(t):
    return t.detach().cpu().numpy()


@pytest.mark.parametrize("prec,solver", [("fp32", "ir"), ("fp32", "gmres"), ("bf16", "ir"), ("fp64", "direct")])
def test_lse_under_poisoned_lds(h, prec, solver):
    note(f"poison lse {prec} {solver} 513x257x65 kappa 1e4")
    P = wl.lse_conditioned(np.random.default_rng(901), 513, 257, 65, 1e4)
    m, n, p = P.shape
    x, r, v = lsq.empty(n), lsq.empty(m), lsq.empty(p)
    rc, res = h.lse_solve(D(P.A), D(P.B), D(P.b), D(P.d), x, r, v, lsq.default_opts(prec=prec, solver=solver))
    assert rc == 0 and res.berr_max <= 1e-14, (rc, res.as_dict())
    xo, ro, vo = direct.lse_solve(P.A, P.B, P.b, P.d)
    cond = direct.lse_cond_x(P.A, P.B, xo, ro, vo)
    assert np.max(np.abs(H(x) - xo)) <= 10 * cond * U64 * np.max(np.abs(xo))


@pytest.mark.parametrize("solver", ["ir", "gmres"])
def test_gls_under_poisoned_lds(h, solver):
    note(f"poison gls fp32 {solver} 300x70x260 kappa 1e5")
    G = wl.gls_conditioned(np.random.default_rng(902), 300, 70, 260, 1e5)
    n, m, p = G.shape
    x, y, z = lsq.empty(m), lsq.empty(p), lsq.empty(n)
    rc, res = h.gls_solve(D(G.W), D(G.V), D(G.d), x, y, z, lsq.default_opts(prec="fp32", solver=solver))
    assert rc == 0 and res.berr_max <= 1e-14, (rc, res.as_dict())
    xo, yo, zo = direct.gls_solve(G.W, G.V, G.d)
    cx, cy = direct.gls_cond_xy(G.W, G.V, xo, yo, zo)
    assert np.max(np.abs(H(x) - xo)) <= 10 * cx * U64 * np.max(np.abs(xo))
    assert np.max(np.abs(H(y) - yo)) <= 10 * cy * U64 * np.max(np.abs(yo))


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_persistent_batch_under_poisoned_lds(h, prec):
    # without the launch-shape table, so that every instance starts on the
    # FP32 (BF16) kernel and the failures reach the FP64 rung beside it
    note(f"poison persistent batch 40 instances, {prec} first")
    probs = list(wl.batch_instances(seed=903, count=40, kappa_max=1e8, m_range=(64, 600)))
    from paper_2406_16499_amd import selector as sel
    ups = [sel._device_problem(P) for P in probs]
    h.batch_tuning([])
    rc, res = h.lsq_solve_batched([d for d, _ in ups], lsq.default_opts(prec=prec, solver="ir"))
    assert rc == 0
    for P, (_, k), r in zip(probs, ups, res):
        assert r.info == 0 and r.berr_max <= 1e-14, r.as_dict()
        x = H(k[1])
        if P.kind == "lse":
            assert direct.lse_err1(P.B, P.d, x) <= 1e-13
        else:
            assert direct.gls_err1(P.W, P.V, P.d, x, H(k[2])) <= 1e-13
