"""The C-ABI library loads on a machine without a GPU and exports every entry point the
header declares (no compute calls)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tpsurf.h")
LIB = os.path.join(ROOT, "paper_2107_01664_amd", "libtpsurf.so")


def declared():
    src = open(HEADER).read()
    return sorted(set(re.findall(r"^TP_API\s+[\w\s\*]+?\b(tp_\w+)\s*\(", src, flags=re.M)))


def test_header_declares_entry_points():
    names = declared()
    for must in ("tp_energy", "tp_gradient", "tp_fractional_apply", "tp_precond_step"):
        assert must in names
    assert len(names) >= 20


def test_library_exports_header_symbols():
    if not os.path.exists(LIB):
        pytest.skip("libtpsurf.so not built")
    L = ctypes.CDLL(LIB)
    missing = [n for n in declared() if not hasattr(L, n)]
    assert not missing, missing


def test_binding_lists_every_symbol():
    from paper_2107_01664_amd import tpsurf
    assert sorted(tpsurf.EXPORTED) == declared()


def test_defaults_without_gpu():
    """tp_params_default / tp_step_opts_default touch no device."""
    if not os.path.exists(LIB):
        pytest.skip("libtpsurf.so not built")
    from paper_2107_01664_amd import tpsurf
    p = tpsurf.default_params()
    assert (p.alpha, p.beta, p.sigma, p.precision, p.cg_rtol, p.cg_maxiter) == (6.0, 12.0, -1.0, 3, 1e-10, 20000)
    assert (p.cg_precond, p.theta, p.leaf_size) == (1, 0.0, 8)
    o = tpsurf.step_opts()
    assert o.line_search == 1 and o.max_backtracks == 30 and o.shrink == 0.5
