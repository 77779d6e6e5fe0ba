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
from ._abi import ORTH_SVQB, ORTH_TSQR, PREC_FP64, PREC_MIXED, ChebfdError, check, load  # noqa: F401

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


def _order_arg(order, n):
    if order is None:
        return None, None
    o = np.ascontiguousarray(order, dtype=np.int32)
    if o.shape != (n,):
        raise ValueError("order must hold n row indices")
    return o, o.ctypes.data_as(ctypes.c_void_p)


def chebfd_matrix_query(rowptr, C=32, sigma=256, prec=PREC_FP64, order=None) -> int:
    rowptr = np.ascontiguousarray(rowptr, dtype=np.int64)
    keep, op = _order_arg(order, len(rowptr) - 1)
    b = ctypes.c_size_t()
    check(load().chebfd_matrix_query(len(rowptr) - 1, rowptr.ctypes.data_as(ctypes.c_void_p), op,
                                     C, sigma, prec, ctypes.byref(b)))
    return b.value


def chebfd_matrix_build(rowptr, col, val, C=32, sigma=256, prec=PREC_FP64, device="cuda", order=None) -> Matrix:
    """Build the device matrix from host CRS arrays (int64 rowptr, int32 col, complex128 val);
    `order` optionally gives the row order (a permutation of 0..n-1) before the sigma sort."""
    rowptr = np.ascontiguousarray(rowptr, dtype=np.int64)
    col = np.ascontiguousarray(col, dtype=np.int32)
    val = np.ascontiguousarray(val, dtype=np.complex128)
    keep, op = _order_arg(order, len(rowptr) - 1)
    nbytes = chebfd_matrix_query(rowptr, C, sigma, prec, order=keep)
    buf = device_buffer(nbytes, device)
    h = _abi.ChebfdMatrix()
    vp = lambda a: a.ctypes.data_as(ctypes.c_void_p)  # noqa: E731
    check(load().chebfd_matrix_build(len(rowptr) - 1, vp(rowptr), vp(col), vp(val), op, C, sigma, prec,
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


def chebfd_random_phase(H: Matrix, m: int, n_b: int, seed: int, col0: int = 0, prec: int | None = None,
                        out=None):
    """Random-phase block (m columns) in the blocked layout (m // n_b, n, n_b), generated on the device."""
    prec = H.prec if prec is None else prec
    if out is None:
        out = torch.empty((m // n_b, H.n, n_b), dtype=vec_dtype(prec), device=H.buf.device)
    check(load().chebfd_random_phase(H.ref(), m, n_b, prec, seed & 0xFFFFFFFFFFFFFFFF,
                                     col0 & 0xFFFFFFFFFFFFFFFF, _ptr(out), _stream()))
    return out


KERNEL_LDS, KERNEL_ROW, KERNEL_MULTIROW, KERNEL_WINDOW = 0, 1, 2, 3
KERNEL_NAMES = {KERNEL_LDS: "lds", KERNEL_ROW: "row", KERNEL_MULTIROW: "multirow", KERNEL_WINDOW: "window"}


def chebfd_step_kernel(H: Matrix, n_b: int) -> int:
    """Which fused-step kernel the filter calls launch for H and n_b (KERNEL_*)."""
    k = ctypes.c_int32()
    check(load().chebfd_step_kernel(H.ref(), n_b, ctypes.byref(k)))
    return k.value


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


def chebfd_filter_unfused(H: Matrix, alpha: float, beta: float, gamma, n_s: int, n_b: int, xy: torch.Tensor,
                          work: FilterWork | None = None, moments: bool = True):
    """chebfd_filter built from separate SpMMV, dot and axpby calls (same arguments and results)."""
    gamma = np.ascontiguousarray(gamma, dtype=np.float64)
    n_p = len(gamma) - 1
    if work is None:
        work = FilterWork(H, n_b, n_p, n_s, moments)
    if xy.dtype != vec_dtype(H.prec) or xy.numel() != H.n * n_s or not xy.is_contiguous():
        raise ValueError("xy must be a contiguous blocked tensor of n * n_s elements in the matrix precision")
    eta = work.eta if moments else None
    nu = work.nu if moments else None
    check(load().chebfd_filter_unfused(H.ref(), alpha, beta, gamma.ctypes.data_as(ctypes.c_void_p), n_p, n_s,
                                       n_b, H.prec, _ptr(xy), _ptr(work.u), _ptr(work.w), _ptr(eta), _ptr(nu),
                                       _ptr(work.work), work.nbytes, _stream()))
    return eta, nu


def chebfd_filter_noalloc(H: Matrix, alpha: float, beta: float, gamma, n_s: int, n_b: int, xy: torch.Tensor,
                          u: torch.Tensor, w: torch.Tensor, eta: torch.Tensor | None, nu: torch.Tensor | None):
    """chebfd_filter with the library's static scratch instead of a workspace; every
    buffer is the caller's (this call allocates nothing)."""
    gamma = np.ascontiguousarray(gamma, dtype=np.float64)
    check(load().chebfd_filter_noalloc(H.ref(), alpha, beta, gamma.ctypes.data_as(ctypes.c_void_p),
                                       len(gamma) - 1, n_s, n_b, H.prec, _ptr(xy), _ptr(u), _ptr(w), _ptr(eta),
                                       _ptr(nu), _stream()))


def chebfd_filter_streamed(H: Matrix, alpha: float, beta: float, gamma, n_s: int, n_b: int, h_xy: torch.Tensor,
                           moments: bool = True, copy_stream=None):
    """Filter the blocked search space h_xy held in (pinned) host memory in place; two
    device staging blocks, copies on `copy_stream` (a new stream if None); returns
    (eta, nu) device tensors or (None, None).  Synchronise torch's current stream
    before reading h_xy."""
    gamma = np.ascontiguousarray(gamma, dtype=np.float64)
    n_p = len(gamma) - 1
    if h_xy.is_cuda or h_xy.dtype != vec_dtype(H.prec) or h_xy.numel() != H.n * n_s or not h_xy.is_contiguous():
        raise ValueError("h_xy must be a contiguous host tensor of n * n_s elements in the matrix precision")
    dev = H.buf.device
    dt = vec_dtype(H.prec)
    u = torch.empty((H.n, n_b), dtype=dt, device=dev)
    w = torch.empty((H.n, n_b), dtype=dt, device=dev)
    sz = ctypes.c_size_t()
    check(load().chebfd_filter_streamed_query(H.ref(), n_p, n_b, ctypes.byref(sz)))
    work = device_buffer(sz.value, dev)
    eta = torch.zeros((n_p + 1, n_s), dtype=torch.complex128, device=dev) if moments else None
    nu = torch.zeros((n_p + 1, n_s), dtype=torch.float64, device=dev) if moments else None
    xs = torch.cuda.Stream(device=dev) if copy_stream is None else copy_stream
    check(load().chebfd_filter_streamed(H.ref(), alpha, beta, gamma.ctypes.data_as(ctypes.c_void_p), n_p, n_s,
                                        n_b, H.prec, ctypes.c_void_p(h_xy.data_ptr()), _ptr(u), _ptr(w), _ptr(eta),
                                        _ptr(nu), _ptr(work), sz.value, _stream(), ctypes.c_void_p(xs.cuda_stream)))
    # keep the device buffers alive until the stream has passed them
    torch.cuda.current_stream().synchronize()
    return eta, nu


def chebfd_op(H: Matrix, alpha: float, beta: float, gamma: float, n_b: int, u, w, y, work: torch.Tensor,
              work_bytes: int):
    check(load().chebfd_op(H.ref(), alpha, beta, gamma, n_b, H.prec, _ptr(u), _ptr(w), _ptr(y),
                           _ptr(work), work_bytes, _stream()))


def chebfd_probe_stream(kind: int, a: torch.Tensor, b: torch.Tensor, c: torch.Tensor | None = None,
                        s: float = 3.0):
    check(load().chebfd_probe_stream(kind, a.numel(), _ptr(b), _ptr(c), s, _ptr(a), _stream()))


def chebfd_spmmv(H: Matrix, alpha: float, beta: float, x: torch.Tensor, y: torch.Tensor | None = None):
    """y = (alpha H + beta I) x for one blocked block x of shape (n, n_b) (or (1, n, n_b))."""
    n_b = x.shape[-1]
    if y is None:
        y = torch.empty_like(x)
    nbytes = chebfd_filter_query(H, n_b)
    work = device_buffer(nbytes, x.device)
    check(load().chebfd_spmmv(H.ref(), alpha, beta, n_b, H.prec, _ptr(x), _ptr(y), _ptr(work), nbytes,
                              _stream()))
    return y


def chebfd_kpm_moments(H: Matrix, alpha: float, beta: float, n_steps: int, R: int, seed: int = 0):
    """Averaged KPM moments mu_0 .. mu_{2 n_steps - 1} of alpha H + beta I from R
    device-drawn random-phase vectors (numpy float64 array)."""
    sz = ctypes.c_size_t()
    check(load().chebfd_kpm_query(H.ref(), n_steps, R, ctypes.byref(sz)))
    work = device_buffer(sz.value, H.buf.device)
    mu = np.empty(2 * n_steps, dtype=np.float64)
    check(load().chebfd_kpm_moments(H.ref(), alpha, beta, n_steps, R, seed,
                                    mu.ctypes.data_as(_abi.DP), _ptr(work), sz.value, _stream()))
    return mu


def chebfd_gram(a: torch.Tensor, b: torch.Tensor, m1: int | None = None, m2: int | None = None):
    """S = A^H B for blocked tensors a (n_blocks, n, n_b) and b of the same precision and n_b."""
    nblk, n, n_b = a.shape
    m1 = nblk * n_b if m1 is None else m1
    m2 = b.shape[0] * n_b if m2 is None else m2
    prec = PREC_FP64 if a.dtype == torch.complex128 else PREC_MIXED
    sz = ctypes.c_size_t()
    check(load().chebfd_gram_query(n, m1, m2, ctypes.byref(sz)))
    work = device_buffer(sz.value, a.device)
    S = torch.zeros((m2, m1), dtype=torch.complex128, device=a.device)   # column-major m1 x m2
    check(load().chebfd_gram(n, n_b, m1, m2, prec, _ptr(a), _ptr(b), _ptr(S), m1, _ptr(work), sz.value,
                             _stream()))
    return S.T


def chebfd_update(a: torch.Tensor, M: torch.Tensor, prec_z: int | None = None):
    """Z = A M for a blocked tensor a (n_blocks, n, n_b) and a complex128 (m1, m2) matrix M."""
    nblk, n, n_b = a.shape
    m1, m2 = M.shape
    prec_a = PREC_FP64 if a.dtype == torch.complex128 else PREC_MIXED
    prec_z = prec_a if prec_z is None else prec_z
    Mc = M.to(torch.complex128).T.contiguous()      # column-major
    z = torch.zeros(((m2 + n_b - 1) // n_b, n, n_b), dtype=vec_dtype(prec_z), device=a.device)
    check(load().chebfd_update(n, n_b, m1, m2, prec_a, _ptr(a), _ptr(Mc), m1, prec_z, _ptr(z), _stream()))
    return z


def chebfd_tsqr(y: torch.Tensor, m: int | None = None):
    """Q, R with y = Q R (TSQR) for a blocked tensor y (n_blocks, n, n_b) holding m columns:
    Q of the same shape and precision, R an (m, m) complex128 upper triangle with a real
    non-negative diagonal."""
    nblk, n, n_b = y.shape
    m = nblk * n_b if m is None else m
    prec = PREC_FP64 if y.dtype == torch.complex128 else PREC_MIXED
    sz = ctypes.c_size_t()
    check(load().chebfd_tsqr_query(n, m, n_b, ctypes.byref(sz)))
    work = device_buffer(sz.value, y.device)
    q = torch.zeros_like(y)
    R = torch.zeros((m, m), dtype=torch.complex128, device=y.device)   # column-major m x m
    check(load().chebfd_tsqr(n, m, n_b, prec, _ptr(y), _ptr(q), _ptr(R), m, _ptr(work), sz.value, _stream()))
    return q, R.T


def chebfd_heev(A: torch.Tensor):
    """Eigenvalues (ascending) and eigenvectors of a Hermitian complex128 CUDA matrix."""
    m = A.shape[0]
    a = A.to(torch.complex128).T.contiguous()        # column-major copy (overwritten)
    v = torch.empty_like(a)
    w = torch.empty(m, dtype=torch.float64, device=A.device)
    sz = ctypes.c_size_t()
    check(load().chebfd_heev_query(m, ctypes.byref(sz)))
    work = device_buffer(sz.value, A.device)
    sweeps = ctypes.c_int32()
    check(load().chebfd_heev(m, _ptr(a), m, _ptr(v), m, _ptr(w), _ptr(work), sz.value, _stream(),
                             ctypes.byref(sweeps)))
    return w, v.T, sweeps.value


class SolveResult:
    def __init__(self, **kw):
        self.__dict__.update(kw)

    def __repr__(self):
        return (f"SolveResult(status={self.status}, iterations={self.stats.iterations}, "
                f"n_found={self.n_found})")


def chebfd_solve(H: Matrix, H64: Matrix, lam_L: float, lam_R: float, n_s: int, n_p: int, n_b: int,
                 tol: float | None = None, max_iter: int = 50, seed: int = 0, x0: torch.Tensor | None = None,
                 spec_bounds=None, want_vectors: bool = True, orth: str = "svqb"):
    """Run the device ChebFD iteration; returns theta, residuals, Ritz vectors (column-major c128).
    orth: "svqb" (SVQB twice) or "tsqr" (rank-revealing TSQR) before each Rayleigh-Ritz step."""
    prec = H.prec
    if tol is None:
        tol = 1e-9 if prec == PREC_FP64 else 1e-7
    p = _abi.ChebfdParams()
    p.lam_L, p.lam_R, p.n_s, p.n_p, p.n_b, p.prec = lam_L, lam_R, n_s, n_p, n_b, prec
    p.tol, p.max_iter, p.seed = tol, max_iter, seed
    p.orth = {"svqb": ORTH_SVQB, "tsqr": ORTH_TSQR}[orth]
    p.spec_lo, p.spec_hi = (float("nan"), float("nan")) if spec_bounds is None else spec_bounds
    sz = ctypes.c_size_t()
    check(load().chebfd_solve_query(H.ref(), H64.ref(), ctypes.byref(p), ctypes.byref(sz)))
    work = device_buffer(sz.value, H.buf.device)
    if x0 is not None:
        _colmajor_ok(x0, H.n)
    Z = torch.empty((n_s, H.n), dtype=torch.complex128, device=H.buf.device).T if want_vectors else None
    theta = np.empty(n_s)
    resid = np.empty(n_s)
    nf = ctypes.c_int32()
    st = _abi.ChebfdStats()
    rc = check(load().chebfd_solve(H.ref(), H64.ref(), ctypes.byref(p), _ptr(x0), _ptr(work), sz.value,
                                   _stream(), ctypes.byref(nf), theta.ctypes.data_as(ctypes.c_void_p),
                                   _ptr(Z), resid.ctypes.data_as(ctypes.c_void_p), ctypes.byref(st)))
    return SolveResult(status=rc, n_found=nf.value, theta=theta, resid=resid, Z=Z, stats=st,
                       workspace_bytes=sz.value)


# ---------------------------------------------------------------------------
# Parameter choice: moment features, heuristic / network -> (n_p, n_s)
# ---------------------------------------------------------------------------
def chebfd_features(H: Matrix, lam_L: float, lam_R: float, seed: int = 0):
    """(features float32[258], count estimate, alpha, beta) of H and [lam_L, lam_R]."""
    sz = ctypes.c_size_t()
    check(load().chebfd_features_query(H.ref(), ctypes.byref(sz)))
    work = device_buffer(sz.value, H.buf.device)
    f = np.empty(_abi.MLP_IN, dtype=np.float32)
    cnt, al, be = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    check(load().chebfd_features(H.ref(), lam_L, lam_R, seed, f.ctypes.data_as(_abi.FP), ctypes.byref(cnt),
                                 ctypes.byref(al), ctypes.byref(be), _ptr(work), sz.value, _stream()))
    return f, cnt.value, al.value, be.value


def chebfd_choose_params(a: float, b: float, count_est: float, n_b: int, mlp_out=None, kappa: float = 1.0,
                         t_mean=(0.0, 0.0), t_std=(1.0, 1.0), t_lo=(0.0, 0.0), t_hi=(0.0, 0.0)):
    """(n_p, n_s) from the heuristic (mlp_out None) or the network's two outputs (host only);
    t_lo, t_hi: the range the de-standardised outputs are held to (unset when equal)."""
    pr = _abi.ChebfdPredictor()
    pr.kappa = kappa
    pr.t_mean[0], pr.t_mean[1] = t_mean
    pr.t_std[0], pr.t_std[1] = t_std
    pr.t_lo[0], pr.t_lo[1] = t_lo
    pr.t_hi[0], pr.t_hi[1] = t_hi
    out = None
    if mlp_out is not None:
        out = np.ascontiguousarray(np.asarray(mlp_out, dtype=np.float32)[:2])
    n_p, n_s = ctypes.c_int32(), ctypes.c_int32()
    check(load().chebfd_choose_params(a, b, count_est, n_b, None if out is None else out.ctypes.data_as(_abi.FP),
                                      ctypes.byref(pr), ctypes.byref(n_p), ctypes.byref(n_s)))
    return n_p.value, n_s.value


def _mlp_work(batch: int, device):
    sz = ctypes.c_size_t()
    check(load().chebfd_mlp_query(batch, None, ctypes.byref(sz)))
    return device_buffer(sz.value, device), sz.value


def _f32(t: torch.Tensor, shape=None):
    assert t.dtype == torch.float32 and t.is_contiguous() and t.is_cuda, "float32 contiguous CUDA tensor expected"
    if shape is not None:
        assert tuple(t.shape) == tuple(shape), (tuple(t.shape), shape)
    return t


def chebfd_mlp_forward(params: torch.Tensor, x: torch.Tensor) -> torch.Tensor:
    """Network outputs (batch, 2) for features x (batch, 258)."""
    _f32(params, (_abi.MLP_PARAMS,))
    batch = x.shape[0]
    _f32(x, (batch, _abi.MLP_IN))
    y = torch.empty((batch, _abi.MLP_OUT), dtype=torch.float32, device=x.device)
    work, nbytes = _mlp_work(batch, x.device)
    check(load().chebfd_mlp_forward(_ptr(params), batch, _ptr(x), _ptr(y), _ptr(work), nbytes, _stream()))
    return y


def chebfd_mlp_grad(params: torch.Tensor, x: torch.Tensor, t: torch.Tensor):
    """(loss (1,), gradient (n_params,)) of sum ||y - t||^2 / (2 batch)."""
    _f32(params, (_abi.MLP_PARAMS,))
    batch = x.shape[0]
    _f32(x, (batch, _abi.MLP_IN))
    _f32(t, (batch, _abi.MLP_OUT))
    loss = torch.empty(1, dtype=torch.float32, device=x.device)
    grad = torch.empty_like(params)
    work, nbytes = _mlp_work(batch, x.device)
    check(load().chebfd_mlp_grad(_ptr(params), batch, _ptr(x), _ptr(t), _ptr(loss), _ptr(grad), _ptr(work),
                                 nbytes, _stream()))
    return loss, grad


def chebfd_mlp_adam(params: torch.Tensor, grad: torch.Tensor, m: torch.Tensor, v: torch.Tensor, step: int,
                    lr: float = 1e-3, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8):
    """One Adam step in place on params, m, v."""
    for t in (params, grad, m, v):
        _f32(t, (_abi.MLP_PARAMS,))
    check(load().chebfd_mlp_adam(_ptr(params), _ptr(grad), _ptr(m), _ptr(v), step, lr, beta1, beta2, eps,
                                 _stream()))
