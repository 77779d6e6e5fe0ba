"""Closed-form spectrum of the clean (W = 0) periodic Topi lattice.

With a Bloch wave e^{i k.s} on every site, the hopping blocks T_d at (s, s+e_d)
and T_d^H at (s, s-e_d) combine into the 4x4 Bloch Hamiltonian

    h(k) = (m - t sum_d cos k_d) G0 - t sum_d sin k_d G_d ,

and because G0..G3 anticommute pairwise and square to one,
h(k)^2 = [(m - t sum_d cos k_d)^2 + t^2 sum_d sin^2 k_d] I.  Each k = 2 pi j / N_d
therefore contributes the eigenvalues +E(k) and -E(k), each twice.  Used as a
pin for the input generator and for solves on clean lattices.
"""
import numpy as np


def bloch_spectrum(Nx: int, Ny: int, Nz: int, m: float, t: float = 1.0) -> np.ndarray:
    ks = [2.0 * np.pi * np.arange(N) / N for N in (Nx, Ny, Nz)]
    kx, ky, kz = np.meshgrid(*ks, indexing="ij")
    a = (m - t * (np.cos(kx) + np.cos(ky) + np.cos(kz))) ** 2 \
        + t * t * (np.sin(kx) ** 2 + np.sin(ky) ** 2 + np.sin(kz) ** 2)
    E = np.sqrt(a.ravel())
    return np.sort(np.concatenate([E, E, -E, -E]))
