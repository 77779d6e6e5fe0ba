"""Algorithmic data volume and flop counts of the Chebyshev filter (Sect. 3.4, Eq. 2).

The paper's minimum-traffic model for one chebfd_op step on a block of n_b
vectors: every matrix entry is loaded once per step (value plus a 4-byte
index; 20 bytes for complex double), and per row and vector U is read once,
W and X are read and written once: 5 vector entries.  Its flop count is 146
per row and vector for the Topi matrices (13 non-zeros per row).
"""
from __future__ import annotations


def value_bytes(prec: int) -> int:
    """Bytes of one stored complex entry: c128 (prec 0) or c64 (prec 1)."""
    return 16 if prec == 0 else 8


def step_bytes(n: int, nnz: int, n_b: int, prec: int) -> tuple[int, int]:
    """(read, write) bytes of one fused step on one block: matrix + U + W + X read, W + X written."""
    s = value_bytes(prec)
    read = nnz * (s + 4) + 3 * n * n_b * s
    write = 2 * n * n_b * s
    return read, write


def start_bytes(n: int, nnz: int, n_b: int, prec: int) -> tuple[int, int]:
    """(read, write) of the two start launches (the start of Alg. 1): U = H~X; W = 2H~U - X, X = ..."""
    s = value_bytes(prec)
    first = (nnz * (s + 4) + n * n_b * s, n * n_b * s)
    second = (nnz * (s + 4) + 2 * n * n_b * s, 2 * n * n_b * s)
    return first[0] + second[0], first[1] + second[1]


def filter_bytes(n: int, nnz: int, n_s: int, n_b: int, n_p: int, prec: int) -> int:
    """Algorithmic bytes of one full filter application (all n_s / n_b blocks, degree n_p >= 2)."""
    r, w = step_bytes(n, nnz, n_b, prec)
    r0, w0 = start_bytes(n, nnz, n_b, prec)
    return (n_s // n_b) * ((n_p - 2) * (r + w) + r0 + w0)


def unfused_step_bytes(n: int, nnz: int, n_b: int, prec: int) -> tuple[int, int]:
    """(read, write) bytes of one recurrence step of the unfused filter, each call
    streaming its operands once: the SpMMV W <- 2(aH+bI)U - W (matrix, U, W read;
    W written), <W, U> (W, U read), <U, U> (U read), X <- X + g W (X, W read; X
    written): 9 vector entries per row and column instead of the fused step's 5."""
    s = value_bytes(prec)
    read = nnz * (s + 4) + 7 * n * n_b * s
    write = 2 * n * n_b * s
    return read, write


def unfused_filter_bytes(n: int, nnz: int, n_s: int, n_b: int, n_p: int, prec: int) -> int:
    """Bytes of the unfused filter (n_p >= 2): the start calls (U = H~X with <U,X>, <X,X>:
    matrix + 5 entries; W <- X, W <- 2H~U - W, <W,U>, <U,U>, X <- g0 X + g1 U, X += g2 W:
    matrix + 14 entries) and n_p - 2 recurrence steps, per block."""
    s = value_bytes(prec)
    r, w = unfused_step_bytes(n, nnz, n_b, prec)
    start = 2 * nnz * (s + 4) + 19 * n * n_b * s
    return (n_s // n_b) * ((n_p - 2) * (r + w) + start)


def filter_flops(n: int, n_s: int, n_p: int, nnzr: float = 13.0) -> float:
    """Flops of one filter with the paper's count, 146 per row and vector per step for
    nnzr = 13 (8 per complex multiply-add of the sparse product plus 42 for the
    recurrence, the dot products and the update)."""
    per = 8.0 * nnzr + 42.0
    return per * n * n_s * n_p


def intensity(n_b: int, nnzr: int = 13, prec: int = 0) -> float:
    """Eq. 2 generalised: flop per byte of one step, 146 / (260 / n_b + 80) for FP64, nnzr = 13."""
    s = value_bytes(prec)
    return (8.0 * nnzr + 42.0) / (nnzr * (s + 4) / n_b + 5 * s)


def roofline(n_b: int, bandwidth_gbs: float, peak_gflops: float = float("inf"), prec: int = 0) -> float:
    """Eq. 1: P* = min(P_max, I(n_b) b) in Gflop/s."""
    return min(peak_gflops, intensity(n_b, prec=prec) * bandwidth_gbs)
