"""Parity of the HIP filter path (through the C ABI) against the FP64 CPU oracle.

Tolerances follow from the arithmetic.  One Chebyshev step adds a local
rounding error of about (nnzr + 4) u relative to the block's magnitude (nnzr
complex FMAs in the sparse product, the recurrence, the update; u the unit
roundoff of the storage/accumulation type).  The three-term recurrence carries
an error made at step k to step p multiplied by U_{p-k}(x), |U_m(cos t)| <=
1/sin t, so with all scaled eigenvalues in [-s, s] the error of T_p x is at
most p (nnzr + 4) u / sqrt(1 - s^2) (coherent accumulation; rounding usually
grows only like sqrt(p)).  The filtered block sums gamma_p T_p x, so its bound is
sum_p |gamma_p| times that.  The dot products sum n such products.
"""
import numpy as np
import pytest
import torch

import oracle as O
from topi import csr_to_dense, diag_csr, random_phase_block, topi_csr

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


def _run_filter(P, H, prec, n_b, n_s, n_p, X, lam=(-0.4, 0.3), C=32, sigma=256, bounds=None):
    M = P.chebfd_matrix_build(*H, C=C, sigma=sigma, prec=prec)
    lo, hi = P.chebfd_bounds(M) if bounds is None else bounds
    al, be, gam = P.chebfd_coefficients(lo, hi, lam[0], lam[1], n_p)
    xb = P.chebfd_pack(M, _to_dev_colmajor(X), n_b)
    eta, nu = P.chebfd_filter(M, al, be, gam, n_s, n_b, xb)
    Y = P.chebfd_unpack(M, xb)
    torch.cuda.synchronize()
    return (Y.cpu().numpy(), eta.cpu().numpy(), nu.cpu().numpy(), al, be, gam, xb)


def test_device_info(P):
    ncu, name = P.chebfd_device_info()
    assert ncu >= 1 and name.startswith("gfx")


@pytest.mark.parametrize("dims,dil,prec", [((4, 4, 3), 0.0, 0), ((5, 3, 3), 0.3, 0), ((5, 3, 3), 0.3, 1)])
def test_bounds_match_oracle(P, dims, dil, prec):
    H = topi_csr(*dims, m=1.0, W=2.0, seed=3, dilution=dil, dilution_seed=5)
    M = P.chebfd_matrix_build(*H, prec=prec)
    lo, hi = P.chebfd_bounds(M)
    rlo, rhi = O.gershgorin_bounds(H)
    tol = 1e-13 if prec == 0 else 1e-5
    assert abs(lo - rlo) <= tol * abs(rlo) and abs(hi - rhi) <= tol * abs(rhi)


def test_coefficients_match_oracle(P):
    al, be, gam = P.chebfd_coefficients(-3.0, 5.0, -0.2, 0.7, 300)
    ral, rbe = O.scale_factors(-3.0, 5.0)
    assert al == pytest.approx(ral, rel=1e-15) and be == pytest.approx(rbe, rel=1e-15)
    assert np.max(np.abs(gam - O.filter_coefficients(-0.2, 0.7, ral, rbe, 300))) < 1e-15


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("C,sigma,dil", [(32, 256, 0.0), (32, 256, 0.35), (4, 64, 0.35), (1, 1, 0.0)])
def test_pack_unpack_roundtrip(P, prec, C, sigma, dil):
    H = topi_csr(5, 3, 3, m=1.0, W=1.0, seed=2, dilution=dil, dilution_seed=1)
    n = len(H[0]) - 1
    M = P.chebfd_matrix_build(*H, C=C, sigma=sigma, prec=prec)
    if dil > 0 and sigma > 1:
        assert M.handle.identity_perm == 0
    X = random_phase_block(n, 16, 4)
    xb = P.chebfd_pack(M, _to_dev_colmajor(X), 8)
    Y = P.chebfd_unpack(M, xb).cpu().numpy()
    if prec == 0:
        assert np.array_equal(Y, X)
    else:
        assert np.max(np.abs(Y - X)) <= EPS32 * 1.01


# (dims, dilution, n_s, n_b, n_p, C, sigma): ragged row counts, several passes,
# non-identity permutations, every supported n_b, degrees 0..3
CASES = [
    ((4, 4, 3), 0.0, 32, 32, 60, 32, 256),
    ((4, 4, 3), 0.0, 16, 4, 41, 32, 256),
    ((5, 3, 3), 0.3, 8, 8, 37, 32, 256),       # n = 180: not a multiple of C
    ((5, 3, 3), 0.3, 4, 1, 25, 4, 64),
    ((3, 3, 3), 0.0, 4, 2, 3, 32, 256),
    ((3, 3, 3), 0.0, 16, 16, 2, 32, 256),
    ((3, 3, 3), 0.0, 64, 64, 1, 32, 256),
    ((3, 3, 3), 0.0, 128, 128, 0, 32, 256),
    ((6, 5, 4), 0.1, 64, 64, 120, 32, 256),
    ((4, 3, 3), 0.0, 256, 128, 30, 16, 32),
]


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("dims,dil,n_s,n_b,n_p,C,sigma", CASES)
def test_filter_parity(P, prec, dims, dil, n_s, n_b, n_p, C, sigma):
    H = topi_csr(*dims, m=1.0, W=1.5, seed=11, dilution=dil, dilution_seed=2)
    n = len(H[0]) - 1
    X = random_phase_block(n, n_s, 17)
    Y, eta, nu, al, be, gam, _ = _run_filter(P, H, prec, n_b, n_s, n_p, X, C=C, sigma=sigma)
    Yr, etar, nur = O.chebyshev_filter(H, al, be, gam, X, n_b)
    s = np.max(np.abs(np.linalg.eigvalsh(csr_to_dense(*H)))) * al
    u = EPS64 if prec == 0 else EPS32
    nnzr = int(np.max(np.diff(H[0])))
    tol_T = _bound(n_p, nnzr, u, s)                  # error bound of T_p x, |x_i| = 1
    tol_Y = max(np.sum(np.abs(gam)), 1.0) * tol_T
    assert np.max(np.abs(Y - Yr)) <= tol_Y, (np.max(np.abs(Y - Yr)), tol_Y)
    if n_p >= 1:
        # |<a, b>| error <= n * (|a| err_b + |b| err_a) with |T_p x| <= 1 entrywise-rms
        tol_m = 2.0 * n * tol_T + n * 4 * u
        assert np.max(np.abs(eta[1:] - etar[1:])) <= tol_m
        assert np.max(np.abs(nu[1:] - nur[1:].real)) <= tol_m


@pytest.mark.parametrize("prec", [0, 1])
def test_filter_deterministic(P, prec):
    H = topi_csr(6, 6, 4, m=1.0, W=1.0, seed=7)
    n = len(H[0]) - 1
    X = random_phase_block(n, 64, 1)
    r1 = _run_filter(P, H, prec, 32, 64, 80, X)
    r2 = _run_filter(P, H, prec, 32, 64, 80, X)
    assert np.array_equal(r1[0], r2[0]) and np.array_equal(r1[1], r2[1]) and np.array_equal(r1[2], r2[2])


@pytest.mark.parametrize("prec", [0, 1])
def test_filter_chebyshev_identity_large(P, prec):
    # H = diag(cos t_j) at the 64x64x32 configuration's dimension (n = 524288),
    # n_b = 32, the benchmark's launch geometry; T_p(cos t) = cos(p t) gives Y for
    # every row in closed form.
    n, n_b, n_s, n_p = 524288, 32, 32, 300
    t = np.linspace(0.2, np.pi - 0.2, n)
    H = diag_csr(np.cos(t))
    X = random_phase_block(n, n_s, 5)
    gam = np.random.default_rng(1).uniform(-1, 1, n_p + 1) / np.arange(1, n_p + 2)
    M = P.chebfd_matrix_build(*H, prec=prec)
    xb = P.chebfd_pack(M, _to_dev_colmajor(X), n_b)
    eta, nu = P.chebfd_filter(M, 1.0, 0.0, gam, n_s, n_b, xb)
    Y = P.chebfd_unpack(M, xb).cpu().numpy()
    f = np.zeros(n)
    for p in range(n_p + 1):
        f += gam[p] * np.cos(p * t)
    u = EPS64 if prec == 0 else EPS32
    tol = np.sum(np.abs(gam)) * _bound(n_p, 1, u, np.cos(0.2))
    assert np.max(np.abs(Y - f[:, None] * X)) <= tol
    # nu_p = sum_i cos^2((p-1) t_i) for unit-modulus x
    nu = nu.cpu().numpy()
    for p in (1, 2, 3, 150, n_p):
        ref = np.sum(np.cos((p - 1) * t) ** 2)
        assert np.max(np.abs(nu[p] - ref)) <= n * 4 * _bound(p, 1, u, np.cos(0.2))


@pytest.mark.parametrize("dims,W,order_kind,prec", [
    ((64, 64, 32), 1.0, "lattice", 0),      # the benchmark's matrix, row order and launch geometry
    ((64, 64, 32), 1.0, "lattice", 1),
    ((64, 64, 32), 1.0, "natural", 0),
    ((128, 128, 64), 1.5, "lattice", 1),    # the 128x128x64 mixed-precision configuration
    ((128, 128, 64), 1.5, "lattice", 0),
])
def test_single_step_full_size_sampled_rows(P, dims, W, order_kind, prec):
    # one chebfd_op step at full size (n_b = 32, SELL-32-256); sampled rows
    # recomputed from the CRS arrays in FP64
    from paper_1803_02156_amd.ordering import lattice_row_order
    H = topi_csr(*dims, m=1.0, W=W, seed=1002)
    n, n_b = len(H[0]) - 1, 32
    order = lattice_row_order(*dims) if order_kind == "lattice" else None
    M = P.chebfd_matrix_build(*H, prec=prec, order=order)
    rng = np.random.default_rng(0)

    def dev(A):   # original-order host block -> the kernel's permuted blocked layout
        return P.chebfd_pack(M, _to_dev_colmajor(A), n_b, prec=prec)[0]

    U = (rng.standard_normal((n, n_b)) + 1j * rng.standard_normal((n, n_b)))
    W0 = (rng.standard_normal((n, n_b)) + 1j * rng.standard_normal((n, n_b)))
    Yh = (rng.standard_normal((n, n_b)) + 1j * rng.standard_normal((n, n_b)))
    if prec == 1:   # the kernel sees the c64-rounded inputs
        U, W0, Yh = (a.astype(np.complex64).astype(np.complex128) for a in (U, W0, Yh))
    u, w, y = dev(U), dev(W0), dev(Yh)
    nbytes = P.chebfd_filter_query(M, n_b)
    work = P.device_buffer(nbytes)
    al, be, g = 0.1333, 0.0, -0.37
    P.chebfd_op(M, al, be, g, n_b, u, w, y, work, nbytes)
    Wg = P.chebfd_unpack(M, w.reshape(1, n, n_b)).cpu().numpy()
    Yg = P.chebfd_unpack(M, y.reshape(1, n, n_b)).cpu().numpy()
    del u, w, y
    rows = np.concatenate([[0, 1, n - 1], rng.integers(0, n, 2000)])
    rowptr, col, val = H
    if prec == 1:
        val = val.astype(np.complex64).astype(np.complex128)
    uu = EPS64 if prec == 0 else EPS32
    for i in rows:
        sl = slice(rowptr[i], rowptr[i + 1])
        hu = al * (val[sl] @ U[col[sl]]) + be * U[i]
        wn = 2 * hu - W0[i]
        scale = np.sum(np.abs(val[sl])[:, None] * np.abs(U[col[sl]]), axis=0) * 2 * al + np.abs(W0[i])
        assert np.all(np.abs(Wg[i] - wn) <= 20 * uu * (scale + 1e-300))
        assert np.all(np.abs(Yg[i] - (Yh[i] + g * wn)) <= 20 * uu * (np.abs(Yh[i]) + abs(g) * scale))


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("which", ["lattice", "random"])
def test_filter_parity_with_row_order(P, prec, which):
    """A caller row order (a symmetric permutation at ingest) changes only the
    rounding order: parity with the oracle, which never sees the order."""
    from paper_1803_02156_amd.ordering import lattice_row_order
    dims = (8, 8, 4)
    H = topi_csr(*dims, m=1.0, W=1.5, seed=21)
    n = len(H[0]) - 1
    order = lattice_row_order(*dims) if which == "lattice" else \
        np.random.default_rng(5).permutation(n).astype(np.int32)
    n_s, n_b, n_p = 64, 32, 50
    X = random_phase_block(n, n_s, 23)
    M = P.chebfd_matrix_build(*H, prec=prec, order=order)
    assert M.handle.identity_perm == 0
    lo, hi = P.chebfd_bounds(M)
    al, be, gam = P.chebfd_coefficients(lo, hi, -0.4, 0.3, n_p)
    xb = P.chebfd_pack(M, _to_dev_colmajor(X), n_b)
    eta, nu = P.chebfd_filter(M, al, be, gam, n_s, n_b, xb)
    Y = P.chebfd_unpack(M, xb).cpu().numpy()
    Yr, etar, nur = O.chebyshev_filter(H, al, be, gam, X, n_b)
    u = EPS64 if prec == 0 else EPS32
    s = np.max(np.abs(np.linalg.eigvalsh(csr_to_dense(*H)))) * al
    bnd = _bound(n_p, 13, u, s) * np.sum(np.abs(gam))
    assert np.max(np.abs(Y - Yr)) <= bnd
    assert np.max(np.abs(nu.cpu().numpy()[1:] - nur[1:])) <= n * _bound(n_p, 13, u, s) * 4


def _csr_from_entries(n, entries):
    """CRS arrays of a Hermitian matrix from (i, j, value) with i <= j (mirrored)."""
    rows = [[] for _ in range(n)]
    for i, j, v in entries:
        rows[i].append((j, v))
        if i != j:
            rows[j].append((i, np.conj(v)))
    rowptr = np.zeros(n + 1, dtype=np.int64)
    col, val = [], []
    for i in range(n):
        for j, v in sorted(rows[i]):
            col.append(j)
            val.append(v)
        rowptr[i + 1] = len(col)
    return rowptr, np.array(col, dtype=np.int32), np.array(val, dtype=np.complex128)


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("case", ["one_row", "empty_rows_C32", "empty_rows_C4", "all_empty_chunk"])
def test_filter_degenerate_matrices(P, prec, case):
    """A 1 x 1 matrix, and matrices with rows that store no entry (whole SELL
    chunks of width 0 among them): the filter must still match the oracle."""
    if case == "one_row":
        H = _csr_from_entries(1, [(0, 0, 0.5)])
        n_b, n_s, C, sigma = 1, 1, 32, 256
    elif case == "all_empty_chunk":
        # rows 0..31 empty (a whole chunk of width 0), rows 32..40 a small chain
        ent = [(i, i + 1, 0.3 + 0.1j) for i in range(32, 40)] + [(i, i, 0.05 * (i - 36)) for i in range(32, 41)]
        H = _csr_from_entries(41, ent)
        n_b, n_s, C, sigma = 4, 8, 32, 1
    else:
        n = 37
        ent = [(i, i, 0.2 * np.sin(i)) for i in range(0, n, 2)]
        ent += [(i, i + 3, 0.25 - 0.15j) for i in range(0, n - 3, 5)]
        H = _csr_from_entries(n, ent)
        n_b, n_s = 4, 8
        C, sigma = (32, 256) if case == "empty_rows_C32" else (4, 1)
    n = len(H[0]) - 1
    assert case == "one_row" or np.any(np.diff(H[0]) == 0)
    n_p = 20
    X = random_phase_block(n, n_s, 3)
    Y, eta, nu, al, be, gam, _ = _run_filter(P, H, prec, n_b, n_s, n_p, X, lam=(-0.3, 0.2), C=C, sigma=sigma,
                                             bounds=(-1.0, 1.0))
    Yr, etar, nur = O.chebyshev_filter(H, al, be, gam, X, n_b)
    u = EPS64 if prec == 0 else EPS32
    tol_T = _bound(n_p, 13, u, 0.9)
    assert np.max(np.abs(Y - Yr)) <= max(np.sum(np.abs(gam)), 1.0) * tol_T
    tol_m = 2.0 * n * tol_T + n * 4 * u
    assert np.max(np.abs(eta[1:] - etar[1:])) <= tol_m
    assert np.max(np.abs(nu[1:] - nur[1:].real)) <= tol_m
