"""Environment overrides of lsq_opts_default (no GPU needed): each variable
changes only its own field, and values that do not parse or lie outside
their range leave the default in place."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

PROBE = """
import json, sys
sys.path.insert(0, %r)
from paper_2406_16499_amd import lsq
o = lsq.default_opts()
print(json.dumps({k: getattr(o, k) for k in ("prec", "solver", "tol", "maxit", "gmres_maxit",
                                            "escalate", "residual", "polish")}))
""" % ROOT


def opts_with(env):
    clean = {k: v for k, v in os.environ.items() if not k.startswith("LSQ_")}
    clean.update(env)
    out = subprocess.run([sys.executable, "-c", PROBE], env=clean, capture_output=True, text=True,
                         timeout=120)
    assert out.returncode == 0, out.stderr
    return json.loads(out.stdout.strip().splitlines()[-1])


@pytest.fixture(scope="module")
def base():
    pytest.importorskip("numpy")
    from paper_2406_16499_amd import lsq
    if not os.path.exists(lsq.LIB_PATH):
        pytest.skip("liblsq.so not built")
    return opts_with({})


def test_defaults(base):
    from paper_2406_16499_amd import lsq
    assert base["prec"] == lsq.PREC["fp32"] and base["solver"] == lsq.SOLVER["ir"]
    assert base["tol"] == 1e-14 and base["escalate"] == 1 and base["residual"] == 0


def test_each_override_changes_its_field(base):
    from paper_2406_16499_amd import lsq
    cases = [({"LSQ_PREC": "bf16"}, "prec", lsq.PREC["bf16"]),
             ({"LSQ_PREC": "auto"}, "prec", lsq.PREC["auto"]),
             ({"LSQ_SOLVER": "gmres"}, "solver", lsq.SOLVER["gmres"]),
             ({"LSQ_TOL": "1e-12"}, "tol", 1e-12),
             ({"LSQ_MAXIT": "7"}, "maxit", 7),
             ({"LSQ_GMRES_MAXIT": "90"}, "gmres_maxit", 90),
             ({"LSQ_ESCALATE": "0"}, "escalate", 0),
             ({"LSQ_RESIDUAL": "1"}, "residual", 1)]
    for env, field, want in cases:
        got = opts_with(env)
        assert got[field] == want, (env, got)
        for k, v in base.items():
            if k != field:
                assert got[k] == v, (env, k)


def test_bad_values_are_ignored(base):
    for env in ({"LSQ_PREC": "fp128"}, {"LSQ_SOLVER": "lu"}, {"LSQ_TOL": "abc"}, {"LSQ_TOL": "-1"},
                {"LSQ_TOL": "nan"}, {"LSQ_MAXIT": "2.5"}, {"LSQ_MAXIT": "-3"}, {"LSQ_GMRES_MAXIT": "0"},
                {"LSQ_ESCALATE": "2"}, {"LSQ_RESIDUAL": "yes"}, {"LSQ_TOL": "1e-12x"}):
        assert opts_with(env) == base, env
