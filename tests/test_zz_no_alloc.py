"""chebfd_filter_noalloc (static scratch, no workspace argument) against
chebfd_filter on the same inputs: two calls in a row, the second smaller, and
the rejection of a launch geometry whose partial sums exceed the static array.
The two entry points run the same kernels in the same order, so the results
must agree bit for bit."""
import numpy as np
import pytest
import torch

from topi import random_phase_block, topi_csr

pytestmark = pytest.mark.gpu

SCRATCH_BYTES = 4 << 20


@pytest.fixture(scope="module")
def P():
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    import paper_1803_02156_amd as P
    P.load()
    return P


def _to_dev_colmajor(X):
    n, m = X.shape
    t = torch.empty((m, n), dtype=torch.complex128, device="cuda")
    t.copy_(torch.from_numpy(np.ascontiguousarray(X.T)))
    return t.T


def _both(P, dims, prec, n_b, n_s, n_p, order=None):
    H = topi_csr(*dims, m=1.0, W=1.5, seed=5)
    n = len(H[0]) - 1
    M = P.chebfd_matrix_build(*H, prec=prec, order=order)
    lo, hi = P.chebfd_bounds(M)
    al, be, gam = P.chebfd_coefficients(lo, hi, -0.4, 0.3, n_p)
    X = random_phase_block(n, n_s, 9)
    xb = P.chebfd_pack(M, _to_dev_colmajor(X), n_b)
    xa = xb.clone()
    eta, nu = P.chebfd_filter(M, al, be, gam, n_s, n_b, xb)
    work = P.FilterWork(M, n_b, n_p, n_s, moments=True)
    P.chebfd_filter_noalloc(M, al, be, gam, n_s, n_b, xa, work.u, work.w, work.eta, work.nu)
    torch.cuda.synchronize()
    assert torch.equal(xa, xb)
    assert torch.equal(work.eta[1:], eta[1:]) and torch.equal(work.nu[1:], nu[1:])
    return M


def test_noalloc_matches_filter_twice(P):
    from paper_1803_02156_amd.ordering import lattice_row_order
    # the benchmark's kernel (window, FP64 n_b = 32), then a smaller LDS-staged c64 case
    _both(P, (16, 16, 8), 0, 32, 64, 50, order=lattice_row_order(16, 16, 8))
    _both(P, (4, 4, 3), 1, 16, 16, 20)


def test_noalloc_rejects_oversized_partials(P):
    H = topi_csr(64, 64, 32, m=1.0, W=1.0, seed=5)
    M = P.chebfd_matrix_build(*H, prec=0)
    n_b = 128
    need = P.chebfd_filter_query(M, n_b)
    print(f"# partial sums for n_b = {n_b}: {need} bytes", flush=True)
    if need <= SCRATCH_BYTES:
        pytest.skip(f"the launch geometry for n_b = {n_b} fits the static scratch ({need} bytes)")
    xb = torch.zeros((1, M.n, n_b), dtype=torch.complex128, device="cuda")
    u, w = torch.zeros_like(xb[0]), torch.zeros_like(xb[0])
    gam = np.ones(3)
    with pytest.raises(P.ChebfdError) as e:
        P.chebfd_filter_noalloc(M, 0.1, 0.0, gam, n_b, n_b, xb, u, w, None, None)
    assert "static scratch" in str(e.value)
    assert torch.count_nonzero(xb) == 0
