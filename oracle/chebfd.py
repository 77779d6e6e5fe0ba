"""ORACLE -- test infrastructure only.

Plain FP64 ChebFD following the paper (Kreutzer et al., arXiv:1803.02156):
the polynomial filter of Sect. 2, Alg. 1 applied blockwise as in Sect. 3.3,
Alg. 2, followed by the orthogonalisation and restart that Sect. 2 names
(SVQB, or TSQR as the alternative) and a Rayleigh-Ritz projection.  The paper defers the window function,
the damping, the restart details and the convergence test to other work;
the readings used for those are stated at each function.

Heavy loops (sparse products, the filter steps) are in ``chebfd_oracle.c``;
small dense steps use numpy's LAPACK routines as library primitives.
"""
from __future__ import annotations

import ctypes
import math
import os

import numpy as np

from . import build as _build

__all__ = [
    "load_library", "gershgorin_bounds", "scale_factors", "window_coefficients",
    "jackson_damping", "filter_coefficients", "spmmv", "chebyshev_filter",
    "kpm_moments", "count_estimate", "choose_params", "svqb", "qr_positive", "qr_orth",
    "rayleigh_ritz", "residual_norms",
    "fix_phases", "chebfd_solve", "SolveResult",
]

_lib = None


def load_library():
    """Load liboracle.so, compiling it with gcc first if it is missing or stale."""
    global _lib
    if _lib is not None:
        return _lib
    path = _build.build(force=False)
    lib = ctypes.CDLL(path)
    P = ctypes.c_void_p
    i64, i32, f64 = ctypes.c_int64, ctypes.c_int32, ctypes.c_double
    lib.orc_spmmv.argtypes = [i64, P, P, P, f64, f64, ctypes.c_int, P, P]
    lib.orc_spmmv.restype = None
    lib.orc_filter.argtypes = [i64, P, P, P, f64, f64, ctypes.c_int, P,
                               ctypes.c_int, ctypes.c_int, P, P, P]
    lib.orc_filter.restype = ctypes.c_int
    lib.orc_num_threads.restype = ctypes.c_int
    lib.orc_set_num_threads.argtypes = [ctypes.c_int]
    lib.orc_set_num_threads.restype = None
    _lib = lib
    return lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _csr(H):
    rowptr, col, val = H
    rowptr = np.ascontiguousarray(rowptr, dtype=np.int64)
    col = np.ascontiguousarray(col, dtype=np.int32)
    val = np.ascontiguousarray(val, dtype=np.complex128)
    return rowptr, col, val


# ---------------------------------------------------------------------------
# Spectral scaling (Alg. 1 uses alpha H + beta I with spectrum inside [-1, 1])
# ---------------------------------------------------------------------------
def gershgorin_bounds(H):
    """Gershgorin interval [min_i (c_i - r_i), max_i (c_i + r_i)] of a Hermitian CSR matrix.

    c_i = Re H_ii, r_i = sum_{j != i} |H_ij|.  It contains the whole spectrum, which
    is what the scaling alpha H + beta I of Alg. 1 needs.
    """
    rowptr, col, val = _csr(H)
    n = len(rowptr) - 1
    rows = np.repeat(np.arange(n, dtype=np.int64), np.diff(rowptr))
    on_diag = col.astype(np.int64) == rows
    c = np.zeros(n)
    np.add.at(c, rows[on_diag], val[on_diag].real)
    r = np.zeros(n)
    np.add.at(r, rows[~on_diag], np.abs(val[~on_diag]))
    return float(np.min(c - r)), float(np.max(c + r))


def scale_factors(lam_lo: float, lam_hi: float):
    """alpha, beta with alpha*lam_lo + beta = -1 and alpha*lam_hi + beta = 1."""
    if not lam_hi > lam_lo:
        raise ValueError("empty spectral interval")
    alpha = 2.0 / (lam_hi - lam_lo)
    beta = -(lam_hi + lam_lo) / (lam_hi - lam_lo)
    return alpha, beta


# ---------------------------------------------------------------------------
# Filter coefficients g_p c_p (the products that weight each T_p x in Alg. 1)
# ---------------------------------------------------------------------------
def window_coefficients(a: float, b: float, n_p: int) -> np.ndarray:
    """Chebyshev coefficients c_0..c_{n_p} of the indicator of [a, b] within [-1, 1].

    The paper's filter is a window function approximated by a polynomial (Sect. 2).
    The coefficients of f = 1_[a,b] are c_p = (2 - delta_p0)/pi int_0^pi f(cos t) cos(pt) dt,
    i.e. with t_a = arccos a, t_b = arccos b:
        c_0 = (t_a - t_b)/pi,   c_p = 2 (sin p t_a - sin p t_b) / (p pi).
    """
    if not (-1.0 <= a < b <= 1.0):
        raise ValueError("window must satisfy -1 <= a < b <= 1")
    ta, tb = np.arccos(a), np.arccos(b)
    p = np.arange(n_p + 1, dtype=np.float64)
    c = np.empty(n_p + 1)
    c[0] = (ta - tb) / np.pi
    pp = p[1:]
    c[1:] = 2.0 * (np.sin(pp * ta) - np.sin(pp * tb)) / (pp * np.pi)
    return c


def jackson_damping(n_p: int) -> np.ndarray:
    """Jackson kernel factors g_0..g_{n_p} for M = n_p + 1 Chebyshev terms.

    g_p = [(M - p + 1) cos(p q) + sin(p q) cot q] / (M + 1),  q = pi/(M + 1)
    (the Jackson kernel of the kernel polynomial method the paper cites for KPM).
    """
    M = n_p + 1
    q = np.pi / (M + 1)
    p = np.arange(n_p + 1, dtype=np.float64)
    return ((M - p + 1) * np.cos(p * q) + np.sin(p * q) / np.tan(q)) / (M + 1)


def filter_coefficients(lam_L: float, lam_R: float, alpha: float, beta: float,
                        n_p: int) -> np.ndarray:
    """gamma_p = g_p c_p for the search interval [lam_L, lam_R] given in H's units."""
    a, b = alpha * lam_L + beta, alpha * lam_R + beta
    if not (-1.0 < a < b < 1.0):
        raise ValueError("search interval not strictly inside the spectral bounds")
    return jackson_damping(n_p) * window_coefficients(a, b, n_p)


# ---------------------------------------------------------------------------
# The filter (Alg. 1 per block, Alg. 2 over blocks)
# ---------------------------------------------------------------------------
def spmmv(H, alpha: float, beta: float, X: np.ndarray) -> np.ndarray:
    """(alpha H + beta I) X for an n x m complex block (Alg. 1's spmmv())."""
    lib = load_library()
    rowptr, col, val = _csr(H)
    n = len(rowptr) - 1
    X = np.asfortranarray(X, dtype=np.complex128)
    m = X.shape[1]
    Y = np.empty((n, m), dtype=np.complex128, order="F")
    lib.orc_spmmv(n, _ptr(rowptr), _ptr(col), _ptr(val), alpha, beta, m, _ptr(X), _ptr(Y))
    return Y


def chebyshev_filter(H, alpha: float, beta: float, gamma: np.ndarray, X: np.ndarray,
                     n_b: int):
    """Apply sum_p gamma_p T_p(alpha H + beta I) to the n x n_s block X, n_b vectors at a time.

    Returns (Y, eta, nu): Y the filtered block; eta, nu of shape (n_p + 1, n_s) with
    eta[p] = <T_p x, T_{p-1} x> and nu[p] = <T_{p-1} x, T_{p-1} x> for p >= 1
    (the dot products of Alg. 1's recurrence step for p >= 3, the same products of the start vectors for
    p = 1, 2), row 0 zero.
    """
    lib = load_library()
    rowptr, col, val = _csr(H)
    n = len(rowptr) - 1
    gamma = np.ascontiguousarray(gamma, dtype=np.float64)
    n_p = len(gamma) - 1
    Y = np.array(X, dtype=np.complex128, order="F", copy=True)
    n_s = Y.shape[1]
    if Y.shape[0] != n or n_b <= 0 or n_s % n_b:
        raise ValueError("bad block shape")
    eta = np.zeros((n_p + 1, n_s), dtype=np.complex128)
    nu = np.zeros((n_p + 1, n_s), dtype=np.complex128)
    rc = lib.orc_filter(n, _ptr(rowptr), _ptr(col), _ptr(val), alpha, beta, n_p,
                        _ptr(gamma), n_s, n_b, _ptr(Y), _ptr(eta), _ptr(nu))
    if rc != 0:
        raise RuntimeError(f"orc_filter failed ({rc})")
    return Y, eta, nu


def kpm_moments(eta: np.ndarray, nu: np.ndarray) -> np.ndarray:
    """Chebyshev moments mu_m = <x, T_m x>, m = 0..2 n_p - 1, per column.

    The filter's dot products give them by the product rule
    T_k T_k = (T_2k + T_0)/2 and T_{k+1} T_k = (T_{2k+1} + T_1)/2:
        mu_0 = nu_1, mu_1 = eta_1, mu_2k = 2 nu_{k+1} - mu_0, mu_{2k+1} = 2 eta_{k+1} - mu_1.
    """
    n_p = eta.shape[0] - 1
    mu = np.empty((2 * n_p,) + eta.shape[1:], dtype=np.complex128)
    mu0, mu1 = nu[1], eta[1]
    mu[0], mu[1] = mu0, mu1
    for k in range(1, n_p):
        mu[2 * k] = 2.0 * nu[k + 1] - mu0
        mu[2 * k + 1] = 2.0 * eta[k + 1] - mu1
    return mu


def count_estimate(mu: np.ndarray, n: int, a: float, b: float) -> float:
    """Stochastic estimate of the number of eigenvalues of the scaled matrix in [a, b].

    mu: (M, R) moments of R random-phase vectors (|x_i| = 1).  The trace of the
    Jackson-damped window polynomial of degree M - 1 is estimated by the mean of
    x^H p(H~) x: n_T = n * sum_m g_m c_m mu~_m with mu~_m = sum_r mu_m^(r) / (n R).
    This is the eigenvalue count that the moments of Alg. 1 are used to monitor.
    """
    M = mu.shape[0]
    mut = np.real(np.sum(mu, axis=1)) / (n * mu.shape[1])
    coef = jackson_damping(M - 1) * window_coefficients(a, b, M - 1)
    return float(n * np.dot(coef, mut))


def choose_params(a: float, b: float, count_est: float, n_b: int, mlp_out=None, kappa: float = 1.0,
                  t_mean=(0.0, 0.0), t_std=(1.0, 1.0), np_min=50, np_max=20000, ns_max=512,
                  t_lo=(0.0, 0.0), t_hi=(0.0, 0.0)):
    """(n_p, n_s) for the scaled interval [a, b] and a count estimate.

    The paper picks n_s a bit above the number of wanted eigenpairs (Sect. 2)
    and n_p around 10^3 for its problems (Sect. 2.1); it gives no rule.  The
    reading used here: the filter's resolution scales like 1 / n_p in the
    scaled variable, so n_p = kappa / delta with delta = (b - a) / 2, and
    n_s = 2 n_hat rounded up to a block.  A network may instead give two
    scale-free ratios, standardised: log(n_p delta) (its own kappa) and
    log(n_s / max(2 n_hat, n_b)) (its factor on the heuristic's n_s), each held
    to [t_lo, t_hi] (the training targets' range) when t_lo < t_hi; n_s then
    stays at least 1.2 n_hat.
    Clamped: n_p in [np_min, np_max], n_s a multiple of n_b in [n_b, ns_max].
    """
    nhat = max(count_est, 0.0)
    delta = (b - a) / 2.0
    if mlp_out is None:
        np_real = kappa / delta
        ns_real = 2.0 * nhat
    else:
        y = [min(30.0, float(mlp_out[k]) * t_std[k] + t_mean[k]) for k in (0, 1)]
        y = [min(t_hi[k], max(t_lo[k], y[k])) if t_lo[k] < t_hi[k] else y[k] for k in (0, 1)]
        np_real = math.exp(y[0]) / delta
        ns_real = max(math.exp(y[1]) * max(2.0 * nhat, n_b), 1.2 * nhat)
    n_p = int(min(np_max, max(np_min, math.floor(np_real + 0.5))))   # halves round up
    n_s = int(math.ceil(ns_real / n_b) * n_b)
    n_s = min(max(n_s, n_b), max(n_b, ns_max // n_b * n_b))
    return n_p, n_s


# ---------------------------------------------------------------------------
# Orthogonalisation, Rayleigh-Ritz, residuals (Sect. 2: SVQB before restart)
# ---------------------------------------------------------------------------
def svqb(Y: np.ndarray, tau: float | None = None):
    """One SVQB step (Stathopoulos and Wu): Q = Y D V L^{-1/2} with D = diag(Y^H Y)^{-1/2}
    and D Y^H Y D = V L V^H.

    Rank revealing: directions whose eigenvalue is below tau * max(L) carry no
    information -- the eigenvalues of an FP64 Gram matrix are only known to
    ~eps * max(L), and data stored with unit roundoff eps_s only resolves singular
    values down to eps_s -- and are dropped.  Default tau = max(100 eps, (10 eps_s)^2)
    with eps = eps_s = 2^-53 (all-FP64 storage).  Returns (Q, n_dropped); Q has
    the kept directions as columns, in ascending order of L.
    """
    if tau is None:
        tau = max(100.0 * 2.0 ** -53, (10.0 * 2.0 ** -53) ** 2)
    S = Y.conj().T @ Y
    d = np.real(np.diag(S)).copy()
    d[d <= 0] = 1.0
    D = 1.0 / np.sqrt(d)
    L, V = np.linalg.eigh((S * D[:, None]) * D[None, :])
    keep = L > tau * L.max()
    Q = (Y * D[None, :]) @ (V[:, keep] / np.sqrt(L[keep])[None, :])
    return Q, int(np.count_nonzero(~keep))


def qr_positive(X: np.ndarray):
    """X = Q R with orthonormal columns in Q and R upper triangular with a real,
    non-negative diagonal: the factorisation TSQR computes (Sect. 2 names TSQR
    as the alternative to SVQB before the restart).  For X of full column rank
    it is unique, so every stable algorithm -- a Householder QR here (LAPACK as a
    library primitive), a reduction tree of Householder QRs on the device --
    reaches the same Q and R up to rounding.  Returns (Q, R)."""
    Q, R = np.linalg.qr(X, mode="reduced")
    d = np.diag(R).copy()
    a = np.abs(d)
    ph = np.ones_like(d)
    ph[a > 0] = d[a > 0] / a[a > 0]
    return Q * ph[None, :], R * ph.conj()[:, None]


def qr_orth(Y: np.ndarray, tau: float | None = None):
    """Rank-revealing orthogonalisation by QR (the TSQR alternative of Sect. 2).

    Y = Q R (qr_positive); column k of Y depends on the columns before it when
    |R_kk|^2 <= tau ||y_k||^2 (its distance to their span is at the level the
    data resolves), and its direction q_k carries no information.  Such
    columns are removed from Y and the rest factorised again, so that no kept
    column was orthogonalised against a direction made of rounding errors.
    tau as in svqb (the same squared relative singular value floor).  Returns
    (Q of the kept columns in their order, n_dropped)."""
    if tau is None:
        tau = max(100.0 * 2.0 ** -53, (10.0 * 2.0 ** -53) ** 2)
    Q, R = qr_positive(Y)
    col2 = np.sum(np.abs(Y) ** 2, axis=0)
    keep = np.abs(np.diag(R)) ** 2 > tau * col2
    if np.all(keep):
        return Q, 0
    return qr_positive(Y[:, keep])[0], int(np.count_nonzero(~keep))


def rayleigh_ritz(H, Q: np.ndarray):
    """Ritz values (ascending) and vectors of H on span(Q), Q orthonormal.

    G = Q^H H Q in H's own units, made exactly Hermitian, G = S diag(theta) S^H,
    Z = Q S.
    """
    Z = spmmv(H, 1.0, 0.0, Q)
    G = Q.conj().T @ Z
    G = 0.5 * (G + G.conj().T)
    theta, S = np.linalg.eigh(G)
    return theta, Q @ S


def fix_phases(Z: np.ndarray) -> np.ndarray:
    """Multiply each column by a unit phase so that its largest-modulus entry is real positive."""
    idx = np.argmax(np.abs(Z), axis=0)
    ph = Z[idx, np.arange(Z.shape[1])]
    ph = ph / np.abs(ph)
    return Z / ph[None, :]


def residual_norms(H, Z: np.ndarray, theta: np.ndarray) -> np.ndarray:
    """r_i = || H z_i - theta_i z_i ||_2 with z_i normalised to unit length."""
    Zn = Z / np.linalg.norm(Z, axis=0)[None, :]
    R = spmmv(H, 1.0, 0.0, Zn) - Zn * theta[None, :]
    return np.linalg.norm(R, axis=0)


class SolveResult:
    def __init__(self, **kw):
        self.__dict__.update(kw)

    def __repr__(self):
        return f"SolveResult(status={self.status}, iterations={self.iterations}, n_found={self.n_found})"


def chebfd_solve(H, lam_L: float, lam_R: float, n_s: int, n_p: int, n_b: int,
                 X0: np.ndarray, tol: float = 1e-9, max_iter: int = 50,
                 refill_seed: int = 0, bounds=None, trace=None, orth: str = "svqb"):
    """Eigenpairs of the Hermitian CSR matrix H with eigenvalues in [lam_L, lam_R].

    Each iteration: filter the block (Alg. 2 / Alg. 1), orthonormalise it by
    SVQB applied twice (orth="svqb") or by one rank-revealing QR (orth="tsqr",
    qr_orth), both rank revealing, Rayleigh-Ritz on the kept directions,
    restart from those Ritz vectors plus fresh random-phase vectors in place of
    the dropped directions (so that unfiltered vectors never enter a
    Rayleigh-Ritz step).

    Convergence: a Ritz pair inside the closed interval is converged when its
    residual is <= tol; the other pairs inside it are unresolved.  Filtering
    shrinks the residual of an unresolved pair that is becoming an eigenpair
    by at least the filter's damping ratio per iteration; a pair whose residual
    has stopped falling is a stable mixture of eigenvectors at or beyond the
    interval's edges (with a residual up to about the distance to them) and
    further filtering will not turn it into an eigenpair.  The solve stops
    (status 0) when the number of converged pairs repeats the previous
    iteration's and the smallest residual of the unresolved pairs did not
    halve since the previous iteration (or none is left); else after max_iter
    iterations (status 1).  A pair is spurious when its residual exceeds half
    the interval width ([theta - r, theta + r] then covers the whole interval:
    it indicates no eigenvalue in it); if, from the second iteration on, the
    number of non-spurious Ritz pairs inside the interval exceeds 3/4 n_s the
    subspace is too small (status 2).  The paper gives none of these rules;
    they are the readings adopted here.  Refill vectors of iteration k are
    random_phase_block(n, d, refill_seed, col0=k n_s).
    Returns the converged pairs first (ascending), then the rest (ascending).
    If `trace` is a list, (iteration, Ritz values, residuals) of every
    iteration are appended to it.
    """
    from topi import random_phase_block

    if orth not in ("svqb", "tsqr"):
        raise ValueError(f"orth must be 'svqb' or 'tsqr', not {orth!r}")
    lo, hi = gershgorin_bounds(H) if bounds is None else bounds
    alpha, beta = scale_factors(lo, hi)
    gamma = filter_coefficients(lam_L, lam_R, alpha, beta, n_p)
    X = np.asfortranarray(X0, dtype=np.complex128)
    n = X.shape[0]
    prev = -1
    count_est = None
    theta = res = Z = None
    status = 1
    it = 0
    dropped = 0
    prev_unres = np.inf
    for it in range(1, max_iter + 1):
        Y, eta, nu = chebyshev_filter(H, alpha, beta, gamma, X, n_b)
        if it == 1:
            mu = kpm_moments(eta, nu)
            count_est = count_estimate(mu, n, alpha * lam_L + beta, alpha * lam_R + beta)
        if orth == "tsqr":
            Q, dropped = qr_orth(Y)
        else:
            Q, d1 = svqb(Y)
            Q, d2 = svqb(Q)
            dropped = d1 + d2
        theta, Z = rayleigh_ritz(H, Q)
        res = residual_norms(H, Z, theta)
        if trace is not None:
            trace.append((it, theta.copy(), res.copy()))
        inwin = (theta >= lam_L) & (theta <= lam_R)
        conv = inwin & (res <= tol)
        spurious = inwin & (res > 0.5 * (lam_R - lam_L))
        cnt = int(np.count_nonzero(conv))
        # too many eigenvalues for the subspace: from the second iteration on, counted on
        # the non-spurious pairs in the interval (a weak first filter scatters Ritz values)
        if it >= 2 and np.count_nonzero(inwin & ~spurious) > 0.75 * n_s:
            status = 2
            break
        # unresolved pairs count as settled once their smallest residual stops falling
        unres = inwin & ~conv
        unres_min = float(np.min(res[unres])) if np.any(unres) else np.inf
        settled = not np.any(unres) or unres_min > 0.5 * prev_unres
        if cnt == prev and settled:
            status = 0
            break
        prev = cnt
        prev_unres = unres_min
        X = Z
        if dropped:
            X = np.concatenate([Z, random_phase_block(n, dropped, refill_seed, col0=it * n_s)], axis=1)
        X = np.asfortranarray(X)
    conv = (theta >= lam_L) & (theta <= lam_R) & (res <= tol)
    order = np.concatenate([np.nonzero(conv)[0], np.nonzero(~conv)[0]])
    return SolveResult(status=status, iterations=it, n_found=int(conv.sum()),
                       theta=theta[order], Z=fix_phases(Z[:, order]), resid=res[order],
                       count_est=count_est, alpha=alpha, beta=beta, gamma=gamma,
                       n_kept=len(theta))
