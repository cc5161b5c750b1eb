"""The C-ABI library loads on the CPU host and exports every declared symbol."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cclr.h")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(cclr_[a-z_]+)\s*\(", src)))


def test_header_declares_the_entry_points():
    names = declared()
    for n in ("cclr_jacobian_right", "cclr_jacobian_left", "cclr_solve_damped", "cclr_response_function"):
        assert n in names


def test_library_exports_every_declared_symbol():
    import paper_2307_14296_amd as cc
    if not os.path.exists(cc.LIB_PATH):
        pytest.skip("libcclr.so not built")
    L = ctypes.CDLL(cc.LIB_PATH)
    for n in declared():
        assert hasattr(L, n), n
    assert set(cc.EXPORTED) == set(declared())


def test_binding_checks_arguments_without_gpu():
    import paper_2307_14296_amd as cc
    if not os.path.exists(cc.LIB_PATH):
        pytest.skip("libcclr.so not built")
    o = cc.cclr_default_options()
    assert o.prec == cc.CCLR_FP64 and o.tol == 1e-10
    # host-side argument checks fire before any device work
    assert cc.lib().cclr_create(1, 5, ctypes.byref(o), ctypes.byref(ctypes.c_void_p())) == cc.CCLR_EINVAL
    assert "o >= 2" in cc.cclr_last_error(None)
    assert cc.lib().cclr_jacobian_right(None, 1, None, None, None, None, None, None) == cc.CCLR_EINVAL
    assert cc.lib().cclr_jacobian_right_noalloc(None, 1, None, None, None, None, None, None) == cc.CCLR_EINVAL
