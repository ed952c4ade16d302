"""CPU checks of the C ABI: the built library loads and exports every entry
point that include/*.h declares (no compute call is made without a GPU)."""
import ctypes
import glob
import os
import re

import pytest

from paper_1102_2878_amd import dfgt

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    names = set()
    for hdr in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(hdr).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"\b(dfgt_[a-z0-9_]+)\s*\(", text):
            names.add(m.group(1))
    return sorted(names)


def test_header_declares_the_boundary():
    syms = declared_symbols()
    for required in ("dfgt_build_tree", "dfgt_gauss_sum", "dfgt_naive_sum", "dfgt_last_error", "dfgt_tree_free",
                     "dfgt_gauss_sum_grad", "dfgt_gauss_sum_backward", "dfgt_lscv_score"):
        assert required in syms


@pytest.mark.parametrize("sym", declared_symbols())
def test_library_exports_symbol(sym):
    L = dfgt.lib()
    assert hasattr(L, sym), f"{sym} declared in include/ but not exported by libdfgt.so"


def test_version_and_error_string_without_gpu():
    L = dfgt.lib()
    assert b"gfx950" in L.dfgt_version()
    assert isinstance(L.dfgt_last_error(), bytes)


def test_invalid_arguments_are_rejected_on_the_host():
    # argument validation happens before any device work, so it runs without a GPU
    L = dfgt.lib()
    h = ctypes.c_void_p()
    rc = L.dfgt_build_tree(None, 10, 2, None, None, ctypes.byref(h))
    assert rc == 1 and b"pts_dev" in L.dfgt_last_error()
    rc = L.dfgt_build_tree(ctypes.c_void_p(16), 10, 33, None, None, ctypes.byref(h))
    assert rc == 1 and b"d must be" in L.dfgt_last_error()
    hv = (ctypes.c_double * 1)(-1.0)
    rc = L.dfgt_naive_sum(ctypes.c_void_p(16), 4, ctypes.c_void_p(16), 4, 2, hv, 1, 0, ctypes.c_void_p(16), None)
    assert rc == 1 and b"bandwidths" in L.dfgt_last_error()


def test_new_entry_points_reject_null_handles():
    L = dfgt.lib()
    hv = (ctypes.c_double * 1)(1.0)
    cv = (ctypes.c_double * 1)()
    rc = L.dfgt_lscv_score(None, hv, 1, 1e-2, 1, None, cv, None, None, None)
    assert rc == 1 and b"NULL" in L.dfgt_last_error()
    rc = L.dfgt_gauss_sum_grad(None, None, hv, 1, 1e-2, None, None, None, None, None, None)
    assert rc == 1 and b"NULL" in L.dfgt_last_error()
    rc = L.dfgt_gauss_sum_backward(None, None, hv, 1, 1e-2, None, None, None, None, None)
    assert rc == 1 and b"NULL" in L.dfgt_last_error()
    rc = L.dfgt_lcv_score(None, hv, 1, 1e-2, None, cv, None, None, None)
    assert rc == 1 and b"NULL" in L.dfgt_last_error()
    rc = L.dfgt_kde_density(None, None, hv, 1, 1e-2, None, None, None, None)
    assert rc == 1 and b"NULL" in L.dfgt_last_error()
    hs = ctypes.c_double()
    rc = L.dfgt_lscv_optimize(None, 0.1, 1.0, 1e-2, 1, 16, 1e-3, None, ctypes.byref(hs), None, None, None)
    assert rc == 1 and b"NULL" in L.dfgt_last_error()
