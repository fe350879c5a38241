"""The C-ABI library: it loads, exports what include/suco.h declares, and its
host-only entry points behave as documented (no GPU needed)."""
import ctypes as C
import os
import re

import pytest

import oracle
import paper_2411_14754_amd as suco

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    txt = open(os.path.join(ROOT, "include", "suco.h")).read()
    return sorted(set(re.findall(r"SUCO_API\s+[\w\s\*]*?\b(suco_\w+)\s*\(", txt)))


def test_header_declares_the_binding_names():
    assert declared_symbols() == sorted(suco.EXPORTED)


def test_library_exports_every_declared_symbol():
    L = C.CDLL(suco.LIB_PATH)
    for name in declared_symbols():
        assert hasattr(L, name), name


def test_version():
    assert suco.lib().suco_version() == 1


@pytest.mark.parametrize("alpha,n", [(0.03, 1_000_000), (0.05, 10_000), (0.01, 1_000_000), (0.02, 10_000_000),
                                     (1e-9, 100), (1.0, 77), (0.0301, 1000), (0.123456, 987_654)])
def test_count_A_matches_oracle(alpha, n):
    assert suco.count_A(alpha, n) == oracle.count_A(alpha, n)


@pytest.mark.parametrize("beta,n,k", [(0.005, 1_000_000, 10), (0.005, 10_000, 10), (0.001, 10_000, 50),
                                      (0.0059, 1000, 1), (1.0, 123, 5), (0.003, 10_000_000, 10)])
def test_count_B_matches_oracle(beta, n, k):
    assert suco.count_B(beta, n, k) == oracle.count_B(beta, n, k)


def test_count_A_float32_alpha_widened():
    # a per-query alpha arrives as float32 and is widened before the product
    import numpy as np
    a32 = float(np.float32(0.05))
    assert suco.count_A(a32, 10_000) == oracle.count_A(a32, 10_000) == 501


def test_errors_before_any_device_work():
    L = suco.lib()
    out = C.c_void_p()
    assert L.suco_build(None, 10, 4, 1, 2, None, None, C.byref(out)) == suco.SUCO_E_INVAL
    assert b"NULL" in L.suco_last_error()
    assert out.value is None
    assert L.suco_query(None, None, 0, 10, 0.1, 0.1, None, None, None) == suco.SUCO_E_STATE
    assert L.suco_index_free(None) == suco.SUCO_OK
    assert L.suco_index_info(None, None, None, None, None) == suco.SUCO_E_STATE
    assert L.suco_rerank(None, None, 1, None, 5, 1, None, None, None) == suco.SUCO_E_STATE
    flags = C.c_int32(-1)
    assert L.suco_index_flags(None, C.byref(flags)) == suco.SUCO_E_STATE and flags.value == -1
    assert L.suco_query_bf16(None, None, 0, 10, 0.1, 0.1, 0, None, None, None, None, None, None) == suco.SUCO_E_STATE
    assert L.suco_query_bf16_debug(None, None, 0, 10, 0.1, 0.1, 0, None, None, None, None, None, None, None, None,
                                   None, None, None) == suco.SUCO_E_STATE
