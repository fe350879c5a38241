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


def test_shape_limits_inval_vs_unsupported():
    # admitted by the problem but past the kernels: SUCO_E_UNSUPPORTED; outside
    # the problem: SUCO_E_INVAL; both before any device work
    L = suco.lib()
    out = C.c_void_p()
    D = C.c_void_p(16)          # never dereferenced: the shape check comes first
    assert L.suco_build(D, 1000, 512, 200, 8, None, None, C.byref(out)) == suco.SUCO_E_UNSUPPORTED
    assert L.suco_build(D, 1000, 512, 300, 8, None, None, C.byref(out)) == suco.SUCO_E_INVAL
    assert L.suco_build(D, 1000, 64, 8, 129, None, None, C.byref(out)) == suco.SUCO_E_UNSUPPORTED
    assert L.suco_build(D, 100, 64, 8, 101, None, None, C.byref(out)) == suco.SUCO_E_INVAL
    assert L.suco_build(D, 0, 64, 8, 1, None, None, C.byref(out)) == suco.SUCO_E_INVAL
    assert out.value is None


def test_count_A_outside_the_unit_interval():
    # a per-query alpha is not checked on the host; the documented reading:
    # above 1, +inf and NaN activate everything, <= 0 activates one point
    assert suco.count_A(float("nan"), 1000) == 1000
    assert suco.count_A(float("inf"), 1000) == 1000
    assert suco.count_A(2.0, 1000) == 1000
    assert suco.count_A(0.0, 1000) == 1
    assert suco.count_A(-0.5, 1000) == 1


def test_index_load_rejects_bad_files_before_device_work(tmp_path):
    import struct
    L = suco.lib()
    out = C.c_void_p()
    missing = str(tmp_path / "missing.suco").encode()
    assert L.suco_index_load(missing, None, None, C.byref(out)) == suco.SUCO_E_INVAL
    assert b"cannot open" in L.suco_last_error()
    bad = tmp_path / "bad.suco"
    bad.write_bytes(b"NOTANIDX" + bytes(56))
    assert L.suco_index_load(str(bad).encode(), None, None, C.byref(out)) == suco.SUCO_E_INVAL
    assert b"not a SuCo index" in L.suco_last_error()
    # a valid header whose file is too short for its shape
    hdr = b"SUCOIDX1" + struct.pack("<IIqiiiiiiQ8x", 1, 64, 100, 8, 2, 4, 0, 0, 0, 0)
    assert len(hdr) == 64
    short = tmp_path / "short.suco"
    short.write_bytes(hdr + bytes(100))
    assert L.suco_index_load(str(short).encode(), None, None, C.byref(out)) == suco.SUCO_E_INVAL
    assert b"expected" in L.suco_last_error()
    # a shape past the kernels in the header
    hdr2 = b"SUCOIDX1" + struct.pack("<IIqiiiiiiQ8x", 1, 64, 1000, 512, 200, 4, 0, 0, 0, 0)
    big = tmp_path / "big.suco"
    big.write_bytes(hdr2)
    assert L.suco_index_load(str(big).encode(), None, None, C.byref(out)) == suco.SUCO_E_UNSUPPORTED
    assert L.suco_index_save(None, missing) == suco.SUCO_E_STATE
    assert L.suco_index_load(None, None, None, C.byref(out)) == suco.SUCO_E_INVAL
    assert out.value is None
