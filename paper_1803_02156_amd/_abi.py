"""ctypes declarations of the libchebfd C ABI (include/chebfd.h)."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libchebfd.so")

OK, NOT_CONVERGED, SUBSPACE_SMALL = 0, 1, 2
EINVAL, EHIP, EWORKSPACE, EINTERVAL, ENUMERIC = -1, -2, -3, -4, -5
PREC_FP64, PREC_MIXED = 0, 1
ORTH_SVQB, ORTH_TSQR = 0, 1
FEATURE_R, FEATURE_MOMENTS = 16, 256
MLP_IN, MLP_HIDDEN, MLP_OUT, MLP_PARAMS = 258, 128, 2, 49922
NP_MIN, NP_MAX = 50, 20000

P = ctypes.c_void_p
i32, i64, f64, sz = ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_size_t


class ChebfdMatrix(ctypes.Structure):
    _fields_ = [
        ("n", i64), ("nnz", i64), ("n_chunks", i64), ("slots", i64),
        ("C", i32), ("sigma", i32), ("prec", i32), ("max_width", i32),
        ("identity_perm", i32), ("uniform_width", i32), ("window_local", i32 * 2),
        ("chunk_off", P), ("chunk_width", P), ("col", P), ("val", P),
        ("perm", P), ("iperm", P),
    ]


class ChebfdParams(ctypes.Structure):
    _fields_ = [
        ("lam_L", f64), ("lam_R", f64), ("n_s", i32), ("n_p", i32), ("n_b", i32), ("prec", i32),
        ("tol", f64), ("max_iter", i32), ("orth", i32), ("seed", ctypes.c_uint64),
        ("spec_lo", f64), ("spec_hi", f64),
    ]


class ChebfdPredictor(ctypes.Structure):
    _fields_ = [("kappa", f64), ("t_mean", f64 * 2), ("t_std", f64 * 2), ("t_lo", f64 * 2), ("t_hi", f64 * 2)]


class ChebfdStats(ctypes.Structure):
    _fields_ = [
        ("iterations", i32), ("n_found", i32), ("n_kept", i32), ("status", i32),
        ("count_est", f64), ("t_total", f64), ("t_filter", f64), ("t_orth", f64), ("t_rr", f64),
        ("t_resid", f64), ("filter_bytes", f64),
    ]


MP = ctypes.POINTER(ChebfdMatrix)
PP = ctypes.POINTER(ChebfdParams)
SP = ctypes.POINTER(ChebfdStats)
DP = ctypes.POINTER(f64)
FP = ctypes.POINTER(ctypes.c_float)

# name -> (restype, argtypes); every symbol the header declares
SIGNATURES = {
    "chebfd_version": (ctypes.c_int, []),
    "chebfd_last_error": (ctypes.c_char_p, []),
    "chebfd_device_info": (ctypes.c_int, [ctypes.POINTER(i32), ctypes.c_char_p, i32]),
    "chebfd_matrix_query": (ctypes.c_int, [i64, P, P, i32, i32, i32, ctypes.POINTER(sz)]),
    "chebfd_matrix_build": (ctypes.c_int, [i64, P, P, P, P, i32, i32, i32, P, sz, P, MP]),
    "chebfd_bounds_query": (ctypes.c_int, [MP, ctypes.POINTER(sz)]),
    "chebfd_bounds": (ctypes.c_int, [MP, P, sz, P, DP, DP]),
    "chebfd_coefficients": (ctypes.c_int, [f64, f64, f64, f64, i32, DP, DP, P]),
    "chebfd_pack": (ctypes.c_int, [MP, i32, i32, i32, P, P, P]),
    "chebfd_unpack": (ctypes.c_int, [MP, i32, i32, i32, P, P, P]),
    "chebfd_random_phase": (ctypes.c_int, [MP, i32, i32, i32, ctypes.c_uint64, ctypes.c_uint64, P, P]),
    "chebfd_filter_query": (ctypes.c_int, [MP, i32, ctypes.POINTER(sz)]),
    "chebfd_step_kernel": (ctypes.c_int, [MP, i32, ctypes.POINTER(i32)]),
    "chebfd_filter": (ctypes.c_int, [MP, f64, f64, P, i32, i32, i32, i32, P, P, P, P, P, P, sz, P]),
    "chebfd_filter_unfused": (ctypes.c_int, [MP, f64, f64, P, i32, i32, i32, i32, P, P, P, P, P, P, sz, P]),
    "chebfd_filter_noalloc": (ctypes.c_int, [MP, f64, f64, P, i32, i32, i32, i32, P, P, P, P, P, P]),
    "chebfd_filter_streamed_query": (ctypes.c_int, [MP, i32, i32, ctypes.POINTER(sz)]),
    "chebfd_filter_streamed": (ctypes.c_int, [MP, f64, f64, P, i32, i32, i32, i32, P, P, P, P, P, P, sz, P, P]),
    "chebfd_op": (ctypes.c_int, [MP, f64, f64, f64, i32, i32, P, P, P, P, sz, P]),
    "chebfd_spmmv": (ctypes.c_int, [MP, f64, f64, i32, i32, P, P, P, sz, P]),
    "chebfd_kpm_query": (ctypes.c_int, [MP, i32, i32, ctypes.POINTER(sz)]),
    "chebfd_kpm_moments": (ctypes.c_int, [MP, f64, f64, i32, i32, ctypes.c_uint64, DP, P, sz, P]),
    "chebfd_gram_query": (ctypes.c_int, [i64, i32, i32, ctypes.POINTER(sz)]),
    "chebfd_gram": (ctypes.c_int, [i64, i32, i32, i32, i32, P, P, P, i32, P, sz, P]),
    "chebfd_update": (ctypes.c_int, [i64, i32, i32, i32, i32, P, P, i32, i32, P, P]),
    "chebfd_tsqr_query": (ctypes.c_int, [i64, i32, i32, ctypes.POINTER(sz)]),
    "chebfd_tsqr": (ctypes.c_int, [i64, i32, i32, i32, P, P, P, i32, P, sz, P]),
    "chebfd_heev_query": (ctypes.c_int, [i32, ctypes.POINTER(sz)]),
    "chebfd_heev": (ctypes.c_int, [i32, P, i32, P, i32, P, P, sz, P, ctypes.POINTER(i32)]),
    "chebfd_solve_query": (ctypes.c_int, [MP, MP, PP, ctypes.POINTER(sz)]),
    "chebfd_solve": (ctypes.c_int, [MP, MP, PP, P, P, sz, P, ctypes.POINTER(i32), P, P, P, SP]),
    "chebfd_features_query": (ctypes.c_int, [MP, ctypes.POINTER(sz)]),
    "chebfd_features": (ctypes.c_int, [MP, f64, f64, ctypes.c_uint64, FP, DP, DP, DP, P, sz, P]),
    "chebfd_choose_params": (ctypes.c_int, [f64, f64, f64, i32, FP, ctypes.POINTER(ChebfdPredictor),
                                            ctypes.POINTER(i32), ctypes.POINTER(i32)]),
    "chebfd_mlp_query": (ctypes.c_int, [i32, ctypes.POINTER(i32), ctypes.POINTER(sz)]),
    "chebfd_mlp_forward": (ctypes.c_int, [P, i32, P, P, P, sz, P]),
    "chebfd_mlp_grad": (ctypes.c_int, [P, i32, P, P, P, P, P, sz, P]),
    "chebfd_mlp_adam": (ctypes.c_int, [P, P, P, P, i32, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                       ctypes.c_float, P]),
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
