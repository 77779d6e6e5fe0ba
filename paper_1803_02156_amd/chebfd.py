"""Thin Python binding of libchebfd: the same calls as include/chebfd.h.

Marshalling only: device memory comes from PyTorch tensors (their data_ptr) and
work is enqueued on torch's current HIP stream; every computation runs in the
library's kernels.  Requires the built libchebfd.so and a GPU.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _abi
from ._abi import PREC_FP64, PREC_MIXED, ChebfdError, check, load  # noqa: F401

_ALIGN = 256


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t: torch.Tensor | None):
    return ctypes.c_void_p(0 if t is None else t.data_ptr())


def device_buffer(nbytes: int, device="cuda") -> torch.Tensor:
    """A 256-byte aligned uint8 device tensor of at least nbytes (torch's caching
    allocator hands out 512-byte aligned blocks)."""
    t = torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)
    assert t.data_ptr() % _ALIGN == 0
    return t


def vec_dtype(prec: int):
    return torch.complex128 if prec == PREC_FP64 else torch.complex64


class Matrix:
    """A built SELL-C-sigma matrix: the C handle plus the device buffer it points into."""

    def __init__(self, handle: _abi.ChebfdMatrix, buf: torch.Tensor):
        self.handle = handle
        self.buf = buf

    @property
    def n(self) -> int:
        return int(self.handle.n)

    @property
    def prec(self) -> int:
        return int(self.handle.prec)

    def ref(self):
        return ctypes.byref(self.handle)


def chebfd_version() -> int:
    return load().chebfd_version()


def chebfd_device_info():
    n = ctypes.c_int32()
    name = ctypes.create_string_buffer(256)
    check(load().chebfd_device_info(ctypes.byref(n), name, 256))
    return n.value, name.value.decode()


def chebfd_matrix_query(rowptr, C=32, sigma=256, prec=PREC_FP64) -> int:
    rowptr = np.ascontiguousarray(rowptr, dtype=np.int64)
    b = ctypes.c_size_t()
    check(load().chebfd_matrix_query(len(rowptr) - 1, rowptr.ctypes.data_as(ctypes.c_void_p),
                                     C, sigma, prec, ctypes.byref(b)))
    return b.value


def chebfd_matrix_build(rowptr, col, val, C=32, sigma=256, prec=PREC_FP64, device="cuda") -> Matrix:
    """Build the device matrix from host CRS arrays (int64 rowptr, int32 col, complex128 val)."""
    rowptr = np.ascontiguousarray(rowptr, dtype=np.int64)
    col = np.ascontiguousarray(col, dtype=np.int32)
    val = np.ascontiguousarray(val, dtype=np.complex128)
    nbytes = chebfd_matrix_query(rowptr, C, sigma, prec)
    buf = device_buffer(nbytes, device)
    h = _abi.ChebfdMatrix()
    vp = lambda a: a.ctypes.data_as(ctypes.c_void_p)  # noqa: E731
    check(load().chebfd_matrix_build(len(rowptr) - 1, vp(rowptr), vp(col), vp(val), C, sigma, prec,
                                     _ptr(buf), nbytes, _stream(), ctypes.byref(h)))
    return Matrix(h, buf)


def chebfd_bounds(H: Matrix):
    b = ctypes.c_size_t()
    check(load().chebfd_bounds_query(H.ref(), ctypes.byref(b)))
    work = device_buffer(b.value)
    lo, hi = ctypes.c_double(), ctypes.c_double()
    check(load().chebfd_bounds(H.ref(), _ptr(work), b.value, _stream(), ctypes.byref(lo), ctypes.byref(hi)))
    return lo.value, hi.value


def chebfd_coefficients(lam_lo, lam_hi, lam_L, lam_R, n_p):
    """(alpha, beta, gamma[n_p + 1]) computed by the library on the host."""
    gam = np.empty(n_p + 1, dtype=np.float64)
    al, be = ctypes.c_double(), ctypes.c_double()
    check(load().chebfd_coefficients(lam_lo, lam_hi, lam_L, lam_R, n_p, ctypes.byref(al),
                                     ctypes.byref(be), gam.ctypes.data_as(ctypes.c_void_p)))
    return al.value, be.value, gam


def _colmajor_ok(x: torch.Tensor, n: int):
    if x.dtype != torch.complex128 or x.dim() != 2 or x.shape[0] != n or x.stride(0) != 1 \
            or x.stride(1) != n or not x.is_cuda:
        raise ValueError("expected a column-major (n, m) complex128 CUDA tensor")


def chebfd_pack(H: Matrix, x: torch.Tensor, n_b: int, prec: int | None = None, out=None):
    """Column-major (n, m) complex128 -> blocked tensor of shape (m // n_b, n, n_b)."""
    prec = H.prec if prec is None else prec
    _colmajor_ok(x, H.n)
    m = x.shape[1]
    if out is None:
        out = torch.empty((m // n_b, H.n, n_b), dtype=vec_dtype(prec), device=x.device)
    check(load().chebfd_pack(H.ref(), m, n_b, prec, _ptr(x), _ptr(out), _stream()))
    return out


def chebfd_unpack(H: Matrix, xb: torch.Tensor, prec: int | None = None, out=None):
    """Blocked (m // n_b, n, n_b) -> column-major (n, m) complex128."""
    prec = H.prec if prec is None else prec
    nblk, n, n_b = xb.shape
    m = nblk * n_b
    if out is None:
        out = torch.empty((m, n), dtype=torch.complex128, device=xb.device).T
    _colmajor_ok(out, H.n)
    check(load().chebfd_unpack(H.ref(), m, n_b, prec, _ptr(xb), _ptr(out), _stream()))
    return out


def chebfd_filter_query(H: Matrix, n_b: int) -> int:
    b = ctypes.c_size_t()
    check(load().chebfd_filter_query(H.ref(), n_b, ctypes.byref(b)))
    return b.value


class FilterWork:
    """Work buffers of chebfd_filter for one (matrix, n_b, n_p, n_s): U, W, partials, moments."""

    def __init__(self, H: Matrix, n_b: int, n_p: int, n_s: int, moments: bool = True):
        dt = vec_dtype(H.prec)
        dev = H.buf.device
        self.u = torch.empty((H.n, n_b), dtype=dt, device=dev)
        self.w = torch.empty((H.n, n_b), dtype=dt, device=dev)
        self.nbytes = chebfd_filter_query(H, n_b)
        self.work = device_buffer(self.nbytes, dev)
        self.eta = torch.zeros((n_p + 1, n_s), dtype=torch.complex128, device=dev) if moments else None
        self.nu = torch.zeros((n_p + 1, n_s), dtype=torch.float64, device=dev) if moments else None


def chebfd_filter(H: Matrix, alpha: float, beta: float, gamma, n_s: int, n_b: int, xy: torch.Tensor,
                  work: FilterWork | None = None, moments: bool = True):
    """Filter the blocked block xy in place; returns (eta, nu) device tensors or (None, None)."""
    gamma = np.ascontiguousarray(gamma, dtype=np.float64)
    n_p = len(gamma) - 1
    if work is None:
        work = FilterWork(H, n_b, n_p, n_s, moments)
    if xy.dtype != vec_dtype(H.prec) or xy.numel() != H.n * n_s or not xy.is_contiguous():
        raise ValueError("xy must be a contiguous blocked tensor of n * n_s elements in the matrix precision")
    eta = work.eta if moments else None
    nu = work.nu if moments else None
    check(load().chebfd_filter(H.ref(), alpha, beta, gamma.ctypes.data_as(ctypes.c_void_p), n_p, n_s,
                               n_b, H.prec, _ptr(xy), _ptr(work.u), _ptr(work.w), _ptr(eta), _ptr(nu),
                               _ptr(work.work), work.nbytes, _stream()))
    return eta, nu


def chebfd_op(H: Matrix, alpha: float, beta: float, gamma: float, n_b: int, u, w, y, work: torch.Tensor,
              work_bytes: int):
    check(load().chebfd_op(H.ref(), alpha, beta, gamma, n_b, H.prec, _ptr(u), _ptr(w), _ptr(y),
                           _ptr(work), work_bytes, _stream()))


def chebfd_probe_stream(kind: int, a: torch.Tensor, b: torch.Tensor, c: torch.Tensor | None = None,
                        s: float = 3.0):
    check(load().chebfd_probe_stream(kind, a.numel(), _ptr(b), _ptr(c), s, _ptr(a), _stream()))
