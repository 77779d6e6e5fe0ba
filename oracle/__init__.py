"""ORACLE -- test infrastructure only.

A plain, slow, obviously correct FP64 CPU implementation of Chebyshev filter
diagonalization (ChebFD) as the paper states it (Sect. 2, Alg. 1; Sect. 3.3,
Alg. 2), used to check the HIP library.  Only ``tests/``, the smoke check
in ``__graft_entry__`` and the CPU-baseline leg of ``bench.py`` may import it.
It shares no code with the HIP path: its only common ground is the seeded
input generator package ``topi``.
"""
from .chebfd import *  # noqa: F401,F403
from .chebfd import __all__  # noqa: F401
