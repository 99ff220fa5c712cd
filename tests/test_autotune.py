"""The batch tuning table: reading it back, and the C-ABI's checks of it
(positive bucket bounds, non-negative routes, shares inside (0, 1))."""
import json

import pytest

from paper_2406_16499_amd import autotune


def test_load_absent_is_empty(tmp_path):
    assert autotune.load(str(tmp_path / "none.json")) == []


def test_load_roundtrip(tmp_path):
    p = tmp_path / "t.json"
    p.write_text(json.dumps({"entries": [
        {"max_dim": 256, "route": 3e5, "fp64_share": 0.25, "solves_per_s": 1.0},
        {"max_dim": 1024, "route": 0.0, "fp64_share": 0.1875},
        {"max_dim": 1024, "route": 0.0, "fp64_share": 0.0625, "pre": 1.0, "esc_max": 0.2}]}))
    assert autotune.load(str(p)) == [(256, 3e5, 0.25, 0.0, 1.0), (1024, 0.0, 0.1875, 0.0, 1.0),
                                     (1024, 0.0, 0.0625, 1.0, 0.2)]


def test_grid_in_range():
    for kappa_max, routes, shares, pres in autotune.REGIMES:
        assert all(0.0 < s < 1.0 for s in shares)
        assert all(r >= 0.0 for r in routes)
        assert all(0.0 <= p <= 8.0 for p in pres)
    kappas = [r[0] for r in autotune.REGIMES]
    assert kappas == sorted(kappas, reverse=True)       # the regime for any escalation first
    his = [hi for _, hi in autotune.BUCKETS]
    assert his == sorted(his) and len(set(his)) == len(his)


@pytest.mark.gpu
def test_table_checks_and_apply():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2406_16499_amd import lsq
    h = lsq.Handle(load_selector=False, load_tuning=False)
    try:
        h.batch_tuning([(256, 3e5, 0.25), (1024, 1e5, 0.125)])
        h.batch_tuning([])
        h.batch_tuning([(1024, 0.0, 0.25), (256, 0.0, 0.25)])     # any order: the smallest cover wins
        h.batch_tuning([(256, 3e5, 0.25, 1.0)])
        h.batch_tuning([(256, 3e5, 0.25, 1.0, 1.0), (256, 3e5, 0.0625, 0.0, 0.1)])
        for bad in ([(256, 0.0, 1.5)], [(256, -1.0, 0.25)], [(0, 0.0, 0.25)], [(256, 0.0, 0.0)],
                    [(256, 0.0, 0.25, -1.0)], [(256, 0.0, 0.25, 9.0)], [(256, 0.0, 0.25, 0.0, -0.1)],
                    [(256, 0.0, 0.25, 0.0, 1.5)]):
            with pytest.raises(RuntimeError):
                h.batch_tuning(bad)
    finally:
        h.close()


def test_committed_table_is_accepted():
    # Handle() installs this table; every entry must pass lsq_batch_tuning's checks
    table = autotune.load()
    assert table, "the measured table ships with the package"
    keys = [(e[0], e[4]) for e in table]
    assert len(set(keys)) == len(keys)
    for max_dim, route, share, pre, esc_max in table:
        assert max_dim >= 1 and route >= 0.0 and 0.0 < share < 1.0 and 0.0 <= pre <= 8.0
        assert 0.0 <= esc_max <= 1.0
    # every bucket has an entry for any regime (a new handle starts there)
    for d in {e[0] for e in table}:
        assert any(e[0] == d and e[4] == 1.0 for e in table)
    assert max(e[0] for e in table) >= 1024          # covers every instance the persistent kernel takes
