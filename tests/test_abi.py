"""The C ABI: every symbol include/chebfd.h declares is exported by libchebfd.so,
the ctypes table matches, and the host-only entry points validate their inputs."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "chebfd.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(chebfd_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    from paper_1803_02156_amd import _abi
    return _abi.load()


def test_every_declared_symbol_is_exported(lib):
    names = _declared()
    assert len(names) >= 10
    for name in names:
        assert hasattr(lib, name), name


def test_binding_table_covers_header():
    from paper_1803_02156_amd import _abi
    assert set(_abi.SIGNATURES) == set(_declared())


def test_version_and_error_string(lib):
    assert lib.chebfd_version() >= 100
    assert isinstance(lib.chebfd_last_error(), bytes)


def test_coefficients_host_side():
    import paper_1803_02156_amd as P
    import oracle as O
    al, be, gam = P.chebfd_coefficients(-7.5, 7.5, -0.05, 0.05, 200)
    assert be == 0.0
    ral, rbe = O.scale_factors(-7.5, 7.5)
    assert np.max(np.abs(gam - O.filter_coefficients(-0.05, 0.05, ral, rbe, 200))) < 1e-15


@pytest.mark.parametrize("interval", [(-8.0, 0.0), (0.1, 0.1), (0.2, -0.2), (-1.0, 7.6)])
def test_coefficients_reject_bad_interval(interval):
    import paper_1803_02156_amd as P
    with pytest.raises(P.ChebfdError) as e:
        P.chebfd_coefficients(-7.5, 7.5, interval[0], interval[1], 10)
    assert e.value.code == -4


def test_coefficients_reject_bad_args(lib):
    g = np.zeros(4)
    a, b = ctypes.c_double(), ctypes.c_double()
    rc = lib.chebfd_coefficients(1.0, 1.0, 0.0, 0.5, 3, ctypes.byref(a), ctypes.byref(b),
                                 g.ctypes.data_as(ctypes.c_void_p))
    assert rc == -1 and b"bounds" in lib.chebfd_last_error()
    rc = lib.chebfd_coefficients(-1.0, 1.0, -0.5, 0.5, -1, ctypes.byref(a), ctypes.byref(b),
                                 g.ctypes.data_as(ctypes.c_void_p))
    assert rc == -1


def test_matrix_query_validation(lib):
    from topi import topi_csr
    rp, col, val = topi_csr(4, 4, 3)
    n = len(rp) - 1
    sz = ctypes.c_size_t()
    p = rp.ctypes.data_as(ctypes.c_void_p)
    assert lib.chebfd_matrix_query(n, p, 32, 256, 0, ctypes.byref(sz)) == 0
    # 13 slots per row, no padding: col + c128 values, plus chunk tables and permutations
    assert sz.value >= n * 13 * (4 + 16) + 8 * n
    assert lib.chebfd_matrix_query(n, p, 32, 256, 1, ctypes.byref(sz)) == 0
    assert lib.chebfd_matrix_query(n, p, 24, 256, 0, ctypes.byref(sz)) == -1   # C not a power of 2
    assert lib.chebfd_matrix_query(n, p, 32, 48, 0, ctypes.byref(sz)) == -1    # sigma not multiple of C
    assert lib.chebfd_matrix_query(n, p, 32, 256, 2, ctypes.byref(sz)) == -1   # bad precision
    assert lib.chebfd_matrix_query(0, p, 32, 256, 0, ctypes.byref(sz)) == -1   # empty matrix
    bad = rp.copy()
    bad[5] = bad[6] + 1
    assert lib.chebfd_matrix_query(n, bad.ctypes.data_as(ctypes.c_void_p), 32, 256, 0, ctypes.byref(sz)) == -1


def test_filter_rejects_null_handle(lib):
    sz = ctypes.c_size_t()
    assert lib.chebfd_filter_query(None, 32, ctypes.byref(sz)) == -1


def test_probe_rejects_bad_args(lib):
    assert lib.chebfd_probe_stream(2, 16, None, None, 1.0, None, None) == -1
    assert lib.chebfd_probe_stream(0, 15, None, None, 1.0, None, None) == -1
