"""ctypes declarations of the libchebfd C ABI (include/chebfd.h)."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libchebfd.so")

OK, NOT_CONVERGED, SUBSPACE_SMALL = 0, 1, 2
EINVAL, EHIP, EWORKSPACE, EINTERVAL, ENUMERIC = -1, -2, -3, -4, -5
PREC_FP64, PREC_MIXED = 0, 1

P = ctypes.c_void_p
i32, i64, f64, sz = ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_size_t


class ChebfdMatrix(ctypes.Structure):
    _fields_ = [
        ("n", i64), ("nnz", i64), ("n_chunks", i64), ("slots", i64),
        ("C", i32), ("sigma", i32), ("prec", i32), ("max_width", i32),
        ("identity_perm", i32), ("uniform_width", i32),
        ("chunk_off", P), ("chunk_width", P), ("col", P), ("val", P),
        ("perm", P), ("iperm", P),
    ]


MP = ctypes.POINTER(ChebfdMatrix)
DP = ctypes.POINTER(f64)

# name -> (restype, argtypes); every symbol the header declares
SIGNATURES = {
    "chebfd_version": (ctypes.c_int, []),
    "chebfd_last_error": (ctypes.c_char_p, []),
    "chebfd_device_info": (ctypes.c_int, [ctypes.POINTER(i32), ctypes.c_char_p, i32]),
    "chebfd_matrix_query": (ctypes.c_int, [i64, P, i32, i32, i32, ctypes.POINTER(sz)]),
    "chebfd_matrix_build": (ctypes.c_int, [i64, P, P, P, i32, i32, i32, P, sz, P, MP]),
    "chebfd_bounds_query": (ctypes.c_int, [MP, ctypes.POINTER(sz)]),
    "chebfd_bounds": (ctypes.c_int, [MP, P, sz, P, DP, DP]),
    "chebfd_coefficients": (ctypes.c_int, [f64, f64, f64, f64, i32, DP, DP, P]),
    "chebfd_pack": (ctypes.c_int, [MP, i32, i32, i32, P, P, P]),
    "chebfd_unpack": (ctypes.c_int, [MP, i32, i32, i32, P, P, P]),
    "chebfd_filter_query": (ctypes.c_int, [MP, i32, ctypes.POINTER(sz)]),
    "chebfd_filter": (ctypes.c_int, [MP, f64, f64, P, i32, i32, i32, i32, P, P, P, P, P, P, sz, P]),
    "chebfd_op": (ctypes.c_int, [MP, f64, f64, f64, i32, i32, P, P, P, P, sz, P]),
    "chebfd_probe_stream": (ctypes.c_int, [i32, i64, P, P, f64, P, P]),
}

_lib = None


def load(path: str = LIB_PATH):
    """Load libchebfd.so; raises if it has not been built (there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(
            f"libchebfd.so not found at {path}: build it with "
            "`python -m paper_1803_02156_amd.build` (hipcc, gfx950)")
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class ChebfdError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"libchebfd error {code}: {msg}")
        self.code = code


def check(rc: int) -> int:
    if rc < 0:
        raise ChebfdError(rc, load().chebfd_last_error().decode())
    return rc
