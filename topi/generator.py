"""Topi-Nx-Ny-Nz Hamiltonians, a diagonal test matrix and random-phase blocks.

Matrix family (paper Sect. 2.1: four degrees of freedom per site of an
Nx x Ny x Nz lattice, n = 4 Nx Ny Nz, 13 complex non-zeros per row, a 3D-stencil
like structure).  The paper defers the model itself to other work; the model
built here is the four-orbital lattice Hamiltonian

    H = sum_s (m + V_s) G0                       on-site block of site s
      + sum_{s,d} [ T_d  at block (s, s+e_d)  +  T_d^H at block (s+e_d, s) ]

with Dirac matrices G0 = sz (x) 1, G1 = sx (x) sx, G2 = sx (x) sy,
G3 = sx (x) sz, hopping T_d = -(t/2) G0 + (i t/2) G_d, periodic boundaries,
and on-site disorder V_s = W (u_s - 1/2) with u_s uniform in [0, 1).

Site numbering s = x + Nx (y + Ny z), matrix row 4 s + o (orbital fastest).
Every row has exactly 13 stored entries when all Nd >= 3 (one diagonal entry,
two per neighbour block); smaller extents merge coinciding neighbours.

All randomness comes from the SplitMix64 counter generator (Steele, Lea and
Flood, "Fast splittable pseudorandom number generators", OOPSLA 2014): the
output for a 64-bit key is a pure function of that key, so any size or slice
can be generated in any order and reproduced bit for bit.
"""
from __future__ import annotations

import numpy as np

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(z) -> np.ndarray:
    """SplitMix64 output function applied to each 64-bit key (wrapping arithmetic)."""
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = z + _GOLDEN
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def uniform01(keys) -> np.ndarray:
    """Uniform doubles in [0, 1): top 53 bits of splitmix64(key) times 2^-53."""
    return (splitmix64(keys) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def _stream(seed: int, tag: int) -> np.uint64:
    """Per-purpose stream base: splitmix64(seed) xor'ed with a small tag and mixed again."""
    base = splitmix64(np.uint64(seed & 0xFFFFFFFFFFFFFFFF))
    return splitmix64(base ^ np.uint64(tag))


def site_disorder(n_sites: int, W: float, seed: int) -> np.ndarray:
    """On-site potential V_s = W (u_s - 1/2), u_s = uniform01(seed xor s)."""
    s = np.arange(n_sites, dtype=np.uint64)
    u = uniform01(np.uint64(seed & 0xFFFFFFFFFFFFFFFF) ^ s)
    return W * (u - 0.5)


# 4x4 Dirac matrices of the model
_SX = np.array([[0, 1], [1, 0]], dtype=np.complex128)
_SY = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
_SZ = np.array([[1, 0], [0, -1]], dtype=np.complex128)
_I2 = np.eye(2, dtype=np.complex128)
G0 = np.kron(_SZ, _I2)
G = [np.kron(_SX, _SX), np.kron(_SX, _SY), np.kron(_SX, _SZ)]


def hopping_block(d: int, t: float) -> np.ndarray:
    """T_d = -(t/2) G0 + (i t/2) G_d, the block at (s, s + e_d)."""
    return -(t / 2) * G0 + (1j * t / 2) * G[d]


def topi_csr(Nx: int, Ny: int, Nz: int, m: float = 1.0, W: float = 0.0,
             t: float = 1.0, seed: int = 0, dilution: float = 0.0,
             dilution_seed: int = 0):
    """CSR arrays (rowptr int64[n+1], col int32[nnz], val complex128[nnz]) of Topi-Nx-Ny-Nz.

    ``dilution`` removes each bond (s, s+e_d) together with its Hermitian
    partner with that probability (key splitmix64 stream of ``dilution_seed``),
    which gives rows of 1..13 entries; 0 keeps the regular 13-per-row matrix.
    Columns are sorted within each row.
    """
    dims = (int(Nx), int(Ny), int(Nz))
    if min(dims) < 1:
        raise ValueError("lattice extents must be >= 1")
    ns = Nx * Ny * Nz
    n = 4 * ns
    s = np.arange(ns, dtype=np.int64)
    coord = [s % Nx, (s // Nx) % Ny, s // (Nx * Ny)]
    stride = [1, Nx, Nx * Ny]
    V = site_disorder(ns, W, seed)

    # per site and orbital a: 13 slots = diagonal + 2 per (direction, sign)
    cols = np.empty((ns, 4, 13), dtype=np.int64)
    vals = np.zeros((ns, 4, 13), dtype=np.complex128)
    keep = np.ones((ns, 4, 13), dtype=bool)
    for a in range(4):
        cols[:, a, 0] = 4 * s + a
        vals[:, a, 0] = (m + V) * G0[a, a].real
    if dilution > 0.0:
        base = _stream(dilution_seed, 0xB0)
        bond_keep = [uniform01(base ^ (np.uint64(3) * s.astype(np.uint64) + np.uint64(d)))
                     >= dilution for d in range(3)]
    slot = 1
    for d in range(3):
        fwd = s + stride[d] * (((coord[d] + 1) % dims[d]) - coord[d])
        bwd = s + stride[d] * (((coord[d] - 1) % dims[d]) - coord[d])
        T = hopping_block(d, t)
        TH = T.conj().T
        for blk, nbr in ((T, fwd), (TH, bwd)):
            for a in range(4):
                nz = np.nonzero(blk[a])[0]
                assert len(nz) == 2
                for k, b in enumerate(nz):
                    cols[:, a, slot + k] = 4 * nbr + b
                    vals[:, a, slot + k] = blk[a, b]
                    if dilution > 0.0:
                        # bond (s, s+e_d) is owned by s; bond (s-e_d, s) by s-e_d
                        keep[:, a, slot + k] = bond_keep[d] if blk is T else bond_keep[d][bwd]
            slot += 2
    cols = cols.reshape(n, 13)
    vals = vals.reshape(n, 13)
    keep = keep.reshape(n, 13)

    if min(dims) >= 3:
        # no two slots of a row name the same column: sort, then drop diluted slots
        sentinel = np.int64(n)
        ckey = np.where(keep, cols, sentinel)
        order = np.argsort(ckey, axis=1, kind="stable")
        cols = np.take_along_axis(ckey, order, axis=1)
        vals = np.take_along_axis(vals, order, axis=1)
        cnt = keep.sum(axis=1)
        rowptr = np.zeros(n + 1, dtype=np.int64)
        np.cumsum(cnt, out=rowptr[1:])
        mask = cols < sentinel
        col = cols[mask].astype(np.int32)
        val = vals[mask]
        return rowptr, col, val

    # small extents: coinciding neighbours are merged by summing (COO -> CSR)
    import scipy.sparse as sp
    r = np.repeat(np.arange(n, dtype=np.int64), 13)[keep.ravel()]
    A = sp.coo_matrix((vals.ravel()[keep.ravel()], (r, cols.ravel()[keep.ravel()])),
                      shape=(n, n)).tocsr()
    A.sum_duplicates()
    A.sort_indices()
    return A.indptr.astype(np.int64), A.indices.astype(np.int32), A.data.astype(np.complex128)


def diag_csr(diag: np.ndarray):
    """CSR arrays of the diagonal matrix diag(d) (one entry per row)."""
    d = np.asarray(diag, dtype=np.complex128)
    n = d.shape[0]
    return (np.arange(n + 1, dtype=np.int64), np.arange(n, dtype=np.int32), d.copy())


def random_phase_block(n: int, m: int, seed: int, col0: int = 0) -> np.ndarray:
    """n x m complex128 block, entry (i, j) = exp(2 pi i u), u = uniform01(k_j xor i).

    k_j = splitmix64(splitmix64(seed) xor (col0 + j)) identifies column col0 + j, so a
    column has the same entries whatever block it is generated in.  Returned in
    column-major order (Fortran), i.e. each vector contiguous.
    """
    base = splitmix64(np.uint64(seed & 0xFFFFFFFFFFFFFFFF))
    out = np.empty((n, m), dtype=np.complex128, order="F")
    i = np.arange(n, dtype=np.uint64)

    def column(j):
        kj = splitmix64(base ^ np.uint64(col0 + j))
        u = uniform01(kj ^ i)
        out[:, j] = np.exp(2j * np.pi * u)

    if n * m < (1 << 22):
        for j in range(m):
            column(j)
    else:
        # columns are independent; numpy releases the GIL inside these loops
        from concurrent.futures import ThreadPoolExecutor
        with ThreadPoolExecutor(max_workers=min(m, 16)) as ex:
            list(ex.map(column, range(m)))
    return out


def csr_to_dense(rowptr, col, val, n=None) -> np.ndarray:
    """Dense complex128 matrix from CSR arrays (small sizes only)."""
    n = len(rowptr) - 1 if n is None else n
    A = np.zeros((n, n), dtype=np.complex128)
    r = np.repeat(np.arange(n), np.diff(rowptr))
    np.add.at(A, (r, col.astype(np.int64)), val)
    return A
