"""CPU checks of the C-ABI boundary: the built library loads and exports
every entry point that include/lsq.h and include/lsq_debug.h declare.  No
compute call is made (there is no GPU here)."""
import ctypes
import os

import pytest

from paper_2406_16499_amd import lsq


def test_headers_declare_the_documented_entry_points():
    names = lsq.header_symbols()
    for required in ("lse_solve", "gls_solve", "lsq_solve_batched", "lse_solve_batched",
                     "gls_solve_batched", "lsq_create", "lsq_destroy", "lsq_set_stream",
                     "lsq_opts_default"):
        assert required in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(lsq.LIB_PATH):
        pytest.skip("liblsq.so not built (run python -m paper_2406_16499_amd.build)")
    lib = ctypes.CDLL(lsq.LIB_PATH)
    missing = [n for n in lsq.header_symbols() if not hasattr(lib, n)]
    assert not missing, missing


def test_opts_defaults_match_the_header():
    if not os.path.exists(lsq.LIB_PATH):
        pytest.skip("liblsq.so not built")
    o = lsq.default_opts()
    assert o.tol == 1e-14 and o.maxit == 40          # Algorithms 2 and 4 default maxit
    assert o.gmres_restart == 30 and o.escalate == 1


def test_ctypes_layouts_match_the_c_header(tmp_path):
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if not cc:
        pytest.skip("no C compiler")
    src = tmp_path / "sz.c"
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "lsq.h"\n'
                   'int main(void){printf("%zu %zu %zu %zu %zu\\n", sizeof(lsq_opts),'
                   ' sizeof(lsq_problem), sizeof(lsq_result), offsetof(lsq_result, berr),'
                   ' offsetof(lsq_problem, x));return 0;}\n')
    exe = tmp_path / "sz"
    inc = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")
    subprocess.run([cc, "-I", inc, str(src), "-o", str(exe)], check=True)
    got = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True,
                                          check=True).stdout.split()]
    assert got == [ctypes.sizeof(lsq.Opts), ctypes.sizeof(lsq.Problem), ctypes.sizeof(lsq.Result),
                   lsq.Result.berr.offset, lsq.Problem.x.offset]


def test_binding_declares_every_entry_point():
    # the ctypes binding sets a signature for exactly the functions the headers declare
    names = set(lsq.header_symbols())
    assert names == set(lsq._SIGS), (sorted(names - set(lsq._SIGS)), sorted(set(lsq._SIGS) - names))
