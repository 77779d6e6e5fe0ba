"""Parity of the window step kernel (the gathered block staged in LDS) with the
FP64 oracle.

The library picks that kernel for FP64 n_b = 32 and c64 n_b = 64 when rows
have at most 13 entries, C = 32 and at least 700 of 1000 stored entries lie
within three 32-row tiles of their row's tile (`window_local`, computed at
ingest); each case below checks that it runs, and covers both instances (every
chunk 13 wide, or ragged widths), a dimension that is not a multiple of the
tile, the halo at workgroup boundaries and all step modes (filter start,
recurrence, moments only).  Tolerances as in test_gpu_filter.py.
"""
import numpy as np
import pytest
import torch

import oracle as O
from topi import csr_to_dense, random_phase_block, topi_csr

pytestmark = pytest.mark.gpu

EPS64 = 2.0 ** -53
EPS32 = 2.0 ** -24


@pytest.fixture(scope="module")
def P():
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    import paper_1803_02156_amd as P
    P.load()
    return P


def _bound(n_p, nnzr, u, s):
    return max(n_p, 1) * (nnzr + 4) * u / np.sqrt(1.0 - s * s)


def _to_dev_colmajor(X):
    n, m = X.shape
    t = torch.empty((m, n), dtype=torch.complex128, device="cuda")
    t.copy_(torch.from_numpy(np.ascontiguousarray(X.T)))
    return t.T


def _order(dims, pencil):
    if pencil is None:
        return None
    from paper_1803_02156_amd.ordering import lattice_row_order
    return lattice_row_order(*dims, pencil=pencil)


def _check_selected(P, M, n_b):
    h = M.handle
    assert h.C == 32 and h.max_width <= 13 and h.window_local[0] >= 700, list(h.window_local)
    assert P.chebfd_step_kernel(M, n_b) == P.KERNEL_WINDOW


CASES = [
    # dims, dilution, pencil, sigma, prec, n_b, n_s, n_p
    ((4, 4, 20), 0.0, None, 256, 0, 32, 64, 60),      # uniform 13-wide chunks, 40 tiles
    ((5, 6, 7), 0.0, None, 256, 0, 32, 32, 45),       # n = 840: ragged last tile
    ((8, 8, 8), 0.0, (4, 4), 256, 0, 32, 32, 40),     # lattice order, 4 x 4 pencils
    ((4, 4, 20), 0.2, None, 1, 0, 32, 32, 40),        # ragged row widths
    ((5, 6, 11), 0.2, None, 1, 1, 64, 64, 60),        # c64, ragged widths
    ((16, 16, 8), 0.0, (4, 4), 256, 1, 64, 64, 40),   # c64, lattice order
    ((4, 4, 20), 0.0, None, 256, 1, 64, 64, 50),      # c64, n_b = 64
    ((5, 6, 7), 0.0, None, 256, 1, 64, 128, 30),
]


@pytest.mark.parametrize("dims,dil,pencil,sigma,prec,n_b,n_s,n_p", CASES)
def test_window_filter_parity(P, dims, dil, pencil, sigma, prec, n_b, n_s, n_p):
    H = topi_csr(*dims, m=1.0, W=1.5, seed=11, dilution=dil, dilution_seed=2)
    n = len(H[0]) - 1
    M = P.chebfd_matrix_build(*H, C=32, sigma=sigma, prec=prec, order=_order(dims, pencil))
    _check_selected(P, M, n_b)
    X = random_phase_block(n, n_s, 17)
    lo, hi = P.chebfd_bounds(M)
    al, be, gam = P.chebfd_coefficients(lo, hi, -0.4, 0.3, n_p)
    xb = P.chebfd_pack(M, _to_dev_colmajor(X), n_b)
    eta, nu = P.chebfd_filter(M, al, be, gam, n_s, n_b, xb)
    Y = P.chebfd_unpack(M, xb).cpu().numpy()
    Yr, etar, nur = O.chebyshev_filter(H, al, be, gam, X, n_b)
    s = np.max(np.abs(np.linalg.eigvalsh(csr_to_dense(*H)))) * al
    u = EPS64 if prec == 0 else EPS32
    nnzr = int(np.max(np.diff(H[0])))
    tol_T = _bound(n_p, nnzr, u, s)
    tol_Y = max(np.sum(np.abs(gam)), 1.0) * tol_T
    assert np.max(np.abs(Y - Yr)) <= tol_Y, (np.max(np.abs(Y - Yr)), tol_Y)
    tol_m = 2.0 * n * tol_T + n * 4 * u
    eta, nu = eta.cpu().numpy(), nu.cpu().numpy()
    assert np.max(np.abs(eta[1:] - etar[1:])) <= tol_m
    assert np.max(np.abs(nu[1:] - nur[1:].real)) <= tol_m


def test_window_locality_matches_definition(P):
    """window_local (entries per 1000 whose permuted column lies in
    [t0 - h TR, t0 + (h + 1) TR) for the tile start t0 of the permuted row; the
    window kernel's halo h is 3 tiles of 32 rows or 1 tile of 64 rows) against
    a recount from the CRS arrays and the handle's permutation."""
    dims = (8, 8, 8)
    H = topi_csr(*dims, m=1.0, W=1.0, seed=5, dilution=0.1, dilution_seed=3)
    rowptr, col, _ = H
    n = len(rowptr) - 1
    M = P.chebfd_matrix_build(*H, prec=0, order=_order(dims, (4, 4)))
    off = M.handle.perm - M.buf.data_ptr()          # perm[new] = old row, inside the matrix buffer
    perm = M.buf[off:off + 4 * n].view(torch.int32).cpu().numpy()
    iperm = np.empty(n, np.int64)
    iperm[perm] = np.arange(n)
    rows = np.repeat(np.arange(n), np.diff(rowptr))
    pr, pc = iperm[rows], iperm[col]
    for v, (tr, h) in enumerate(((32, 3), (64, 1))):
        t0 = pr // tr * tr
        inside = np.count_nonzero((pc >= t0 - h * tr) & (pc < t0 + (h + 1) * tr))
        assert M.handle.window_local[v] == inside * 1000 // len(col)


@pytest.mark.parametrize("prec,R", [(0, 32), (1, 64)])
def test_window_kpm_moments(P, prec, R):
    # moments-only steps (no Y update) through the window kernel
    H = topi_csr(4, 4, 20, m=1.0, W=1.5, seed=31)
    n = len(H[0]) - 1
    n_steps = 60
    lo, hi = O.gershgorin_bounds(H)
    alpha, beta = O.scale_factors(lo, hi)
    M = P.chebfd_matrix_build(*H, prec=prec)
    _check_selected(P, M, R)
    mu = P.chebfd_kpm_moments(M, alpha, beta, n_steps, R, seed=17)
    X = random_phase_block(n, R, 17)
    _, eta, nu = O.chebyshev_filter(H, alpha, beta, np.zeros(n_steps + 1), X, R)
    ref = np.real(np.sum(O.kpm_moments(eta, nu), axis=1)) / (n * R)
    u = EPS64 if prec == 0 else EPS32
    assert abs(mu[0] - 1.0) < 10 * u
    assert np.max(np.abs(mu - ref)) < 50 * u * n_steps


@pytest.mark.parametrize("prec,n_b", [(0, 32), (1, 64)])
def test_window_filter_deterministic(P, prec, n_b):
    H = topi_csr(4, 4, 20, m=1.0, W=1.0, seed=7)
    n = len(H[0]) - 1
    X = random_phase_block(n, 64, 1)
    out = []
    for _ in range(2):
        M = P.chebfd_matrix_build(*H, prec=prec)
        _check_selected(P, M, n_b)
        lo, hi = P.chebfd_bounds(M)
        al, be, gam = P.chebfd_coefficients(lo, hi, -0.3, 0.3, 70)
        xb = P.chebfd_pack(M, _to_dev_colmajor(X), n_b)
        eta, nu = P.chebfd_filter(M, al, be, gam, 64, n_b, xb)
        out.append((P.chebfd_unpack(M, xb).cpu().numpy(), eta.cpu().numpy(), nu.cpu().numpy()))
    for a, b in zip(*out):
        assert np.array_equal(a, b)


def test_window_selection_rules(P):
    """The window kernel only where it has an instance and the gathers are local."""
    from paper_1803_02156_amd.ordering import lattice_row_order
    dims = (16, 16, 8)
    H = topi_csr(*dims, m=1.0, W=1.0, seed=3)
    M44 = P.chebfd_matrix_build(*H, prec=0, order=lattice_row_order(*dims, pencil=(4, 4)))
    M84 = P.chebfd_matrix_build(*H, prec=0, order=lattice_row_order(*dims, pencil=(8, 4)))
    assert M84.handle.window_local[0] < 700       # z-neighbours 128 rows away
    assert P.chebfd_step_kernel(M44, 32) == P.KERNEL_WINDOW
    assert P.chebfd_step_kernel(M84, 32) == P.KERNEL_LDS
    assert P.chebfd_step_kernel(M44, 16) == P.KERNEL_LDS
    M32 = P.chebfd_matrix_build(*H, prec=1, order=lattice_row_order(*dims, pencil=(4, 4)))
    assert P.chebfd_step_kernel(M32, 64) == P.KERNEL_WINDOW
    assert P.chebfd_step_kernel(M32, 32) == P.KERNEL_LDS
    Hs = topi_csr(3, 3, 3, m=1.0, W=1.0, seed=3)   # 4 tiles: too few for a sweep
    assert P.chebfd_step_kernel(P.chebfd_matrix_build(*Hs, prec=0), 32) == P.KERNEL_LDS
