"""CPU-side checks of the C-ABI library: it loads, exports every function the
header declares, and its host-only paths (argument validation, the Neuberger
coefficients) behave -- no GPU needed, nothing is launched."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "msb.h")
LIB = os.path.join(ROOT, "paper_1010_2592_amd", "_lib", "libmsb.so")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?(?:int|void|char)\s*\*?\s*(\w+)\s*\(", src, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(LIB):
        pytest.fail("libmsb.so is not built (run python -m paper_1010_2592_amd.build)")
    return ctypes.CDLL(LIB)


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("wilson_apply", "mshift_bicgstabl", "mshift_cg", "pfe_sign_apply", "pfe_sign_backward",
              "msb_low_modes", "pfe_sign_apply_deflated",
              "msb_create", "msb_destroy", "msb_last_error"):
        assert n in names


def test_every_declared_symbol_is_exported(L):
    for n in declared_functions():
        assert hasattr(L, n), n


def test_neuberger_matches_oracle(L):
    from oracle import pfe
    for n in (1, 10, 30, 58):
        s = np.zeros(n)
        w = np.zeros(n)
        dp = ctypes.POINTER(ctypes.c_double)
        L.msb_neuberger_pfe.argtypes = [ctypes.c_int, dp, dp]
        assert L.msb_neuberger_pfe(n, s.ctypes.data_as(dp), w.ctypes.data_as(dp)) == 0
        so, wo = pfe.neuberger(n)
        assert np.allclose(s, so, rtol=1e-14) and np.allclose(w, wo, rtol=1e-14)


def test_argument_errors_need_no_gpu(L):
    L.msb_last_error.restype = ctypes.c_char_p
    L.msb_create.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    assert L.msb_create(None, None, None, None) == 1
    assert b"null" in L.msb_last_error()
    dp = ctypes.POINTER(ctypes.c_double)
    L.mshift_bicgstabl.argtypes = [ctypes.c_void_p, ctypes.c_double, ctypes.c_int, dp, dp,
                                   ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_int,
                                   ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                                   ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    s = np.ones(3)
    rc = L.mshift_bicgstabl(None, 1.0, 3, s.ctypes.data_as(dp), s.ctypes.data_as(dp), 0, 2, 1e-8,
                            10, 1, 0, 1, None, None, None, None)
    assert rc == 1 and b"null context" in L.msb_last_error()
    L.msb_neuberger_pfe.argtypes = [ctypes.c_int, dp, dp]
    assert L.msb_neuberger_pfe(0, s.ctypes.data_as(dp), s.ctypes.data_as(dp)) == 1


def test_python_binding_exposes_c_names():
    from paper_1010_2592_amd import msb
    for n in ("wilson_apply", "mshift_bicgstabl", "mshift_cg", "pfe_sign_apply", "pfe_sign_backward"):
        assert callable(getattr(msb, n))
    s, w = msb.neuberger_pfe(10)
    assert s.shape == (10,) and np.all(s > 0)
