"""Pins for the seeded input generator (Topi Hamiltonians, random-phase blocks)."""
import numpy as np
import pytest

from topi import (csr_to_dense, diag_csr, random_phase_block, site_disorder,
                  splitmix64, topi_csr, uniform01)
from topi.generator import G, G0, hopping_block
from tests.bloch import bloch_spectrum


def test_splitmix64_known_answers():
    # the first outputs of a SplitMix64 generator whose state starts at 0
    # (state advances by the golden-ratio increment before each mix)
    inc = 0x9E3779B97F4A7C15
    assert int(splitmix64(np.uint64(0))) == 0xE220A8397B1DCDAF
    assert int(splitmix64(np.uint64(inc))) == 0x6E789E6AA1B965F4
    assert int(splitmix64(np.uint64((2 * inc) % 2 ** 64))) == 0x06C45D188009454F


def test_uniform01_range_and_mean():
    u = uniform01(np.arange(200000, dtype=np.uint64))
    assert u.min() >= 0.0 and u.max() < 1.0
    assert abs(u.mean() - 0.5) < 4 * np.sqrt(1 / 12 / u.size)


def test_dirac_matrices_anticommute():
    mats = [G0] + G
    for i, A in enumerate(mats):
        assert np.allclose(A @ A, np.eye(4))
        assert np.allclose(A, A.conj().T)
        for B in mats[i + 1:]:
            assert np.allclose(A @ B + B @ A, 0)


@pytest.mark.parametrize("dims", [(4, 4, 3), (3, 5, 4)])
def test_topi_structure(dims):
    rp, col, val = topi_csr(*dims, m=1.0, W=2.0, seed=11)
    n = 4 * np.prod(dims)
    assert len(rp) == n + 1
    assert np.all(np.diff(rp) == 13)          # Sect. 2.1: 13 non-zeros per row
    A = csr_to_dense(rp, col, val)
    assert np.array_equal(A, A.conj().T)       # Hermitian, exactly
    for i in range(0, n, 7):                    # columns sorted within rows
        c = col[rp[i]:rp[i + 1]]
        assert np.all(np.diff(c) > 0)


def test_topi_hopping_orientation():
    # block (s, s + e_x) holds T_x, block (s + e_x, s) holds T_x^H
    Nx, Ny, Nz = 4, 3, 3
    A = csr_to_dense(*topi_csr(Nx, Ny, Nz, m=0.7, W=0.0, t=1.3))
    s, sp = 5, 6   # x = 1 -> x = 2 at y = 1, z = 0
    T = hopping_block(0, 1.3)
    assert np.allclose(A[4 * s:4 * s + 4, 4 * sp:4 * sp + 4], T)
    assert np.allclose(A[4 * sp:4 * sp + 4, 4 * s:4 * s + 4], T.conj().T)
    # z hop with periodic wrap: z = Nz-1 -> z = 0
    s = 1 + Nx * (2 + Ny * (Nz - 1))
    sp = 1 + Nx * 2
    assert np.allclose(A[4 * s:4 * s + 4, 4 * sp:4 * sp + 4], hopping_block(2, 1.3))


def test_topi_disorder_on_diagonal():
    Nx, Ny, Nz = 3, 3, 3
    rp, col, val = topi_csr(Nx, Ny, Nz, m=1.0, W=1.5, seed=77)
    A = csr_to_dense(rp, col, val)
    V = site_disorder(27, 1.5, 77)
    d = np.real(np.diag(A)).reshape(27, 4)
    assert np.allclose(d, (1.0 + V)[:, None] * np.array([1, 1, -1, -1])[None, :])
    assert np.all(np.abs(V) <= 0.75)


@pytest.mark.parametrize("dims,m", [((4, 4, 3), 1.0), ((5, 3, 4), 1.7), ((6, 6, 4), 1.0)])
def test_topi_clean_matches_bloch(dims, m):
    A = csr_to_dense(*topi_csr(*dims, m=m, W=0.0))
    e = np.linalg.eigvalsh(A)
    assert np.max(np.abs(e - bloch_spectrum(*dims, m))) < 1e-12


def test_topi_chiral_and_kramers():
    # S = 1 (x) (sy (x) 1) anticommutes with every H of the family
    dims = (4, 4, 3)
    A = csr_to_dense(*topi_csr(*dims, m=1.0, W=2.0, seed=3))
    ns = int(np.prod(dims))
    sy = np.array([[0, -1j], [1j, 0]])
    S = np.kron(np.eye(ns), np.kron(sy, np.eye(2)))
    assert np.allclose(S @ A @ S, -A, atol=1e-14)
    e = np.linalg.eigvalsh(A)
    assert np.allclose(e, -e[::-1], atol=1e-12)           # +- symmetric spectrum
    assert np.allclose(e[0::2], e[1::2], atol=1e-10)       # Kramers pairs


def test_topi_small_extents_merge():
    rp, col, val = topi_csr(2, 3, 1, m=1.0, W=1.0, seed=1)
    A = csr_to_dense(rp, col, val)
    assert np.array_equal(A, A.conj().T)
    assert np.all(np.diff(rp) == 8)


def test_topi_dilution_ragged_hermitian():
    rp, col, val = topi_csr(4, 4, 3, m=1.0, W=1.0, seed=2, dilution=0.3, dilution_seed=9)
    A = csr_to_dense(rp, col, val)
    assert np.array_equal(A, A.conj().T)
    lens = np.diff(rp)
    assert lens.min() < 13 and lens.max() == 13 and np.all(lens % 2 == 1)


def test_random_phase_block():
    X = random_phase_block(1000, 5, 42)
    assert np.allclose(np.abs(X), 1.0)
    # a column does not depend on the block it is generated in
    Y = random_phase_block(1000, 3, 42, col0=2)
    assert np.array_equal(X[:, 2:], Y)
    assert abs(np.mean(X)) < 0.1
    Z = random_phase_block(1000, 5, 43)
    assert not np.allclose(X, Z)


def test_diag_csr():
    rp, col, val = diag_csr(np.array([1.0, -2.0, 0.5]))
    assert np.array_equal(csr_to_dense(rp, col, val), np.diag([1.0, -2.0, 0.5]).astype(complex))


def test_plane_waves_are_eigenvectors_of_the_clean_lattice():
    """The Bloch vectors of the full-size GPU test: H x = E x for the clean lattice."""
    import scipy.sparse as sp
    from tests.test_gpu_fullsize import _bloch_matrix, _plane_wave
    dims = (5, 4, 6)
    H = topi_csr(*dims, m=1.0, W=0.0)
    n = len(H[0]) - 1
    A = sp.csr_matrix((H[2], H[1], H[0]), shape=(n, n))
    rng = np.random.default_rng(3)
    for _ in range(6):
        j = [int(rng.integers(0, N)) for N in dims]
        E, V = np.linalg.eigh(_bloch_matrix([2 * np.pi * jj / N for jj, N in zip(j, dims)]))
        for b in range(4):
            x = _plane_wave(dims, j, V[:, b])
            assert np.max(np.abs(A @ x - E[b] * x)) < 1e-13
