"""The C-ABI library loads on the CPU and exports every entry point of include/schurilu.h."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "schurilu.h")
LIB = os.path.join(ROOT, "paper_2303_08881_amd", "libschurilu.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\**\s*([a-z_][a-z0-9_]*)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for f in ("ilu_setup", "ilu_apply", "fgmres_solve", "ilu_destroy", "ilu_export", "ilu_last_error", "csr_spmv"):
        assert f in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libschurilu.so not built (run __graft_entry__.build())")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [f for f in declared_functions() if not hasattr(lib, f)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="libschurilu.so not built")
def test_default_options_without_gpu():
    import paper_2303_08881_amd as silu
    from paper_2303_08881_amd.binding import _Opts

    o = _Opts()
    silu.lib().ilu_default_options(ctypes.byref(o))
    assert (o.method, o.interior_fact, o.inner_iters, o.pivot_mode) == (silu.BJ, silu.ILU0, 3, silu.PIVOT_ERROR)
    assert (o.trsv_mode, o.factor_prec) == (silu.TRSV_AUTO, silu.PREC_F64)
    assert (o.smooth_fact, o.arnoldi_mode, o.block_split) == (silu.ILU0, silu.ARNOLDI_AUTO, 0)
