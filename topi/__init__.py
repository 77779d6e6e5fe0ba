"""Seeded synthetic inputs shared by the CPU oracle and the GPU path.

This package generates inputs only: the Topi-Nx-Ny-Nz lattice Hamiltonians of the
paper's problem setting (Sect. 2.1), a diagonal test matrix, and random-phase
block vectors.  It holds none of the filter method's arithmetic (no scaling, no
coefficients, no recurrence), so that the oracle and the HIP path share nothing
but their inputs.
"""
from .generator import (  # noqa: F401
    splitmix64,
    uniform01,
    site_disorder,
    topi_csr,
    diag_csr,
    random_phase_block,
    csr_to_dense,
)
