"""The unfused filter (SpMMV, dot and axpby as separate calls) and the step
kernels for general sparse Hermitian matrices, against the FP64 oracle.

* chebfd_filter_unfused: Alg. 1 from separate calls (the paper's GHOST-nofuse
  comparison, Sect. 3.2) must give the same Y, eta and nu as the oracle, for
  each step kernel the library can pick.
* Rows wider than 16 entries or chunks of C = 64 rows (a general Hermitian
  matrix in CRS, Sect. 3.1) are served by the row-per-wavefront kernel
  (n_b >= 32) and the multi-row kernel (n_b < 32): oracle parity on random
  sparse Hermitian matrices with 20..40 entries per row.

Tolerances as in test_gpu_filter.py.
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


def random_hermitian(n, lo, hi, seed):
    """CRS arrays of a random sparse Hermitian matrix: row i gets lo..hi entries
    (i, j) and their mirror images (j, i), so rows hold about 2 lo..2 hi entries;
    real diagonal; columns sorted."""
    import scipy.sparse as sp
    rng = np.random.default_rng(seed)
    k = rng.integers(lo, hi + 1, n)
    r = np.repeat(np.arange(n), k)
    c = rng.integers(0, n, len(r))
    v = rng.uniform(-1, 1, len(r)) + 1j * rng.uniform(-1, 1, len(r))
    A = sp.coo_matrix((v, (r, c)), shape=(n, n)).tocsr()
    Hm = (A + A.conj().T).tocsr()
    Hm = Hm + sp.diags(rng.uniform(-1, 1, n))
    Hm.sum_duplicates()
    Hm.sort_indices()
    return Hm.indptr.astype(np.int64), Hm.indices.astype(np.int32), Hm.data.astype(np.complex128)


def _filter_and_compare(P, H, prec, n_b, n_s, n_p, C, sigma, want_kind, unfused, lam=(-0.4, 0.3), order=None):
    n = len(H[0]) - 1
    M = P.chebfd_matrix_build(*H, C=C, sigma=sigma, prec=prec, order=order)
    assert P.chebfd_step_kernel(M, n_b) == want_kind
    lo, hi = P.chebfd_bounds(M)
    al, be, gam = P.chebfd_coefficients(lo, hi, lam[0], lam[1], n_p)
    X = random_phase_block(n, n_s, 29)
    xb = P.chebfd_pack(M, _to_dev_colmajor(X), n_b)
    run = P.chebfd_filter_unfused if unfused else P.chebfd_filter
    eta, nu = run(M, al, be, gam, n_s, n_b, xb)
    Y = P.chebfd_unpack(M, xb).cpu().numpy()
    eta, nu = eta.cpu().numpy(), nu.cpu().numpy()
    Yr, etar, nur = O.chebyshev_filter(H, al, be, gam, X, n_b)
    s = np.max(np.abs(np.linalg.eigvalsh(csr_to_dense(*H)))) * al + abs(be)
    u = EPS64 if prec == 0 else EPS32
    nnzr = int(np.max(np.diff(H[0])))
    tol_T = _bound(n_p, nnzr, u, min(s, 0.999))
    tol_Y = max(np.sum(np.abs(gam)), 1.0) * tol_T
    assert np.max(np.abs(Y - Yr)) <= tol_Y, (np.max(np.abs(Y - Yr)), tol_Y)
    if n_p >= 1:   # (degree 0 forms no moments)
        tol_m = 2.0 * n * tol_T + n * 4 * u
        assert np.max(np.abs(eta[1:] - etar[1:])) <= tol_m
        assert np.max(np.abs(nu[1:] - nur[1:].real)) <= tol_m
    return Y, eta, nu


# (dims, prec, n_b, n_s, n_p, kernel kind): the Topi cases pick the window and
# LDS-staged kernels, the wide random matrices the row and multi-row kernels
UNFUSED_TOPI = [
    ((4, 4, 20), 0, 32, 64, 40, "window"),
    ((4, 4, 20), 1, 64, 64, 40, "window"),
    ((5, 3, 3), 0, 8, 16, 37, "lds"),
    ((5, 3, 3), 1, 32, 32, 25, "lds"),
    ((3, 3, 3), 0, 4, 8, 2, "lds"),
    ((3, 3, 3), 1, 4, 4, 1, "lds"),
    ((3, 3, 3), 0, 16, 16, 0, "lds"),
]

KINDS = {"window": 3, "lds": 0, "row": 1, "multirow": 2}


@pytest.mark.parametrize("dims,prec,n_b,n_s,n_p,kind", UNFUSED_TOPI)
def test_unfused_filter_matches_oracle_topi(P, dims, prec, n_b, n_s, n_p, kind):
    H = topi_csr(*dims, m=1.0, W=1.5, seed=11)
    _filter_and_compare(P, H, prec, n_b, n_s, n_p, 32, 256, KINDS[kind], unfused=True)


WIDE = [
    # n, entries per row and mirror, C, prec, n_b, n_s, n_p, kernel
    (1500, (10, 20), 64, 0, 32, 64, 30, "row"),
    (1500, (10, 20), 64, 1, 32, 32, 30, "row"),
    (1037, (10, 20), 32, 0, 8, 16, 25, "multirow"),
    (1037, (10, 20), 64, 1, 8, 8, 25, "multirow"),
    (777, (12, 18), 64, 0, 64, 64, 20, "row"),
    (777, (12, 18), 64, 1, 128, 128, 12, "row"),
    (500, (10, 20), 16, 0, 1, 4, 15, "multirow"),
]


@pytest.mark.parametrize("unfused", [False, True])
@pytest.mark.parametrize("n,ent,C,prec,n_b,n_s,n_p,kind", WIDE)
def test_wide_rows_match_oracle(P, n, ent, C, prec, n_b, n_s, n_p, kind, unfused):
    H = random_hermitian(n, *ent, seed=n + C)
    w = np.diff(H[0])
    assert w.max() > 16 and w.min() >= 10
    _filter_and_compare(P, H, prec, n_b, n_s, n_p, C, 256, KINDS[kind], unfused=unfused)


@pytest.mark.parametrize("prec,n_b", [(0, 32), (1, 64), (1, 32)])
def test_unfused_equals_fused_lattice_order(P, prec, n_b):
    """Fused and unfused filters on the same lattice-ordered blocks (the benchmark's
    row order and kernels), both against the oracle."""
    from paper_1803_02156_amd.ordering import lattice_row_order
    dims = (16, 16, 8)
    H = topi_csr(*dims, m=1.0, W=1.0, seed=3)
    order = lattice_row_order(*dims)
    kind = KINDS["window" if (prec, n_b) != (1, 32) else "lds"]
    for unfused in (False, True):
        _filter_and_compare(P, H, prec, n_b, 2 * n_b, 60, 32, 256, kind, unfused=unfused, order=order)
