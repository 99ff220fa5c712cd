"""CPU checks of bench.py's command-line contract: one GPU only (a request
for more exits with status 2 and a message), every workload name parses, and
the source hash that guards the stored hardware-counter summaries is stable."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


@pytest.mark.parametrize("workload", ["lse-large", "gls-large", "lse-wide", "gls-tall", "paper-grid",
                                      "lse-factored", "batched"])
def test_workloads_parse(workload, monkeypatch):
    import bench
    monkeypatch.setattr(sys, "argv", ["bench.py", "--workload", workload, "--steps", "1"])
    a = bench.parse()
    assert a.workload == workload and a.gpus == 1 and a.steps == 1


def test_source_hash_is_stable():
    # bench.py drops a stored hardware-counter figure when this hash differs
    # from the one its summary under profiles/ records
    import bench
    h1, h2 = bench.source_hash(None), bench.source_hash(None)
    assert h1 == h2 and len(h1) == 16
    assert bench.source_hash(bench.BATCH_SOURCES) != h1
