"""The filter on a search space held in pinned host memory (chebfd_filter_streamed,
working sets beyond HBM, Sect. 3.5): the blocks pass through two device staging
blocks while the next one is copied in on a second stream.  Each block is
filtered by chebfd_filter itself, so Y, eta and nu must equal chebfd_filter's
on the device-resident block bit for bit; the first case is also checked
against the FP64 oracle."""
import numpy as np
import pytest
import torch

import oracle as O
from topi import csr_to_dense, random_phase_block, topi_csr

pytestmark = pytest.mark.gpu

EPS64 = 2.0 ** -53


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


@pytest.mark.parametrize("dims,prec,n_b,n_s,n_p", [
    ((6, 6, 4), 0, 32, 128, 40),      # 4 blocks: both staging slots reused
    ((8, 8, 8), 1, 32, 96, 60),       # c64, odd number of blocks
    ((4, 4, 3), 0, 16, 16, 25),       # one block
    ((4, 4, 3), 0, 8, 24, 1),         # degree 1
])
def test_streamed_equals_device_filter(P, dims, prec, n_b, n_s, n_p):
    H = topi_csr(*dims, m=1.0, W=1.5, seed=8)
    n = len(H[0]) - 1
    M = P.chebfd_matrix_build(*H, prec=prec)
    lo, hi = P.chebfd_bounds(M)
    al, be, gam = P.chebfd_coefficients(lo, hi, -0.4, 0.3, n_p)
    X = random_phase_block(n, n_s, 13)
    xb = P.chebfd_pack(M, _to_dev_colmajor(X), n_b)
    h = torch.empty(xb.shape, dtype=xb.dtype, pin_memory=True)
    h.copy_(xb)
    eta, nu = P.chebfd_filter(M, al, be, gam, n_s, n_b, xb)
    eta, nu = eta.clone(), nu.clone()
    eta2, nu2 = P.chebfd_filter_streamed(M, al, be, gam, n_s, n_b, h)
    torch.cuda.synchronize()
    assert torch.equal(h, xb.cpu())
    assert torch.equal(eta2[1:], eta[1:]) and torch.equal(nu2[1:], nu[1:])
    if prec == 0 and n_p == 40:
        Yr, etar, nur = O.chebyshev_filter(H, al, be, gam, X, n_b)
        Y = P.chebfd_unpack(M, h.cuda()).cpu().numpy()
        sc = np.max(np.abs(np.linalg.eigvalsh(csr_to_dense(*H)))) * al + abs(be)
        tol = max(np.sum(np.abs(gam)), 1.0) * n_p * 17 * EPS64 / np.sqrt(1.0 - sc * sc)
        assert np.max(np.abs(Y - Yr)) <= tol
