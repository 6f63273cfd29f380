"""The C-ABI library loads and exports every symbol include/ifmm.h declares
(no compute call: this runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1407_1572_amd", "libifmm.so")
HDR = os.path.join(ROOT, "include", "ifmm.h")


def declared_symbols():
    txt = open(HDR).read()
    return sorted(set(re.findall(r"\b(ifmm_[a-z_]+)\s*\(", txt)))


def test_header_declares_the_boundary():
    syms = declared_symbols()
    for s in ("ifmm_factor", "ifmm_solve", "ifmm_matvec", "ifmm_stats", "ifmm_destroy",
              "ifmm_status_string", "ifmm_diagonal", "ifmm_ranks"):
        assert s in syms


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    for s in declared_symbols():
        assert hasattr(lib, s), s
    lib.ifmm_status_string.restype = ctypes.c_char_p
    assert lib.ifmm_status_string(3) == b"singular pivot block"


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_invalid_arguments_are_rejected_before_any_device_work():
    lib = ctypes.CDLL(LIB)
    h = ctypes.c_void_p()

    class K(ctypes.Structure):
        _fields_ = [("kind", ctypes.c_int), ("ell", ctypes.c_double), ("diag_mode", ctypes.c_int),
                    ("c0", ctypes.c_double), ("diag", ctypes.c_void_p)]

    k = K(0, 0.0, 0, 1.0, None)
    f = lib.ifmm_factor
    f.restype = ctypes.c_int
    P = ctypes.c_void_p
    f.argtypes = [P, ctypes.c_int64, ctypes.POINTER(K), ctypes.c_double, ctypes.c_int, ctypes.c_int,
                  P, P, ctypes.POINTER(P)]
    dummy = P(16)  # never dereferenced: validation fails first
    assert f(dummy, 4096, ctypes.byref(k), 1e-6, 32, 15, None, None, ctypes.byref(h)) == 1  # rank not square
    assert f(dummy, 4096, ctypes.byref(k), -1.0, 32, 16, None, None, ctypes.byref(h)) == 1  # eps < 0
    assert f(dummy, 4096, ctypes.byref(k), 1e-6, 0, 16, None, None, ctypes.byref(h)) == 1   # leaf size
    assert f(dummy, 8, ctypes.byref(k), 1e-6, 32, 16, None, None, ctypes.byref(h)) == 1     # too small
    assert f(dummy, 4096, ctypes.byref(k), 1e-6, 32, 81, None, None, ctypes.byref(h)) == 1  # p > 8
    k2 = K(1, 0.0, 1, 1.0, None)  # exp with ell = 0
    assert f(dummy, 4096, ctypes.byref(k2), 1e-6, 32, 16, None, None, ctypes.byref(h)) == 1
    k3 = K(1, 0.1, 2, 0.0, None)  # diagonal vector without the vector
    assert f(dummy, 4096, ctypes.byref(k3), 1e-6, 32, 16, None, None, ctypes.byref(h)) == 1
    k4 = K(1, 0.1, 7, 1.0, None)  # unknown diagonal rule
    assert f(dummy, 4096, ctypes.byref(k4), 1e-6, 32, 16, None, None, ctypes.byref(h)) == 1
    # eps = 0 (lossless) without an explicit rank cap
    assert f(dummy, 4096, ctypes.byref(k), 0.0, 32, 16, None, None, ctypes.byref(h)) == 1
    lib.ifmm_solve.restype = ctypes.c_int
    assert lib.ifmm_solve(None, None, None, 1, None, None) == 1


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_batched_entry_points_reject_bad_arguments():
    lib = ctypes.CDLL(LIB)
    P = ctypes.c_void_p
    f = lib.ifmm_factor_batched
    f.restype = ctypes.c_int
    assert f(0, None, None, None, ctypes.c_double(1e-8), 64, 36, None, 4, None, None, None) == 1  # count 0
    assert f(3, None, None, None, ctypes.c_double(1e-8), 64, 36, None, 4, None, None, None) == 1  # null arrays
    g = lib.ifmm_solve_batched
    g.restype = ctypes.c_int
    assert g(0, None, None, None, 1, 4, None, None, None) == 1
    assert g(2, None, None, None, 1, 4, None, None, None) == 1
