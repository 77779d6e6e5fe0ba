"""MI355X-native Chebyshev filter diagonalization (ChebFD).

The compute path is libchebfd.so (HIP kernels for gfx950 behind the C ABI of
include/chebfd.h); ``paper_1803_02156_amd.chebfd`` is its Python binding.
"""
from . import _abi  # noqa: F401
from .chebfd import *  # noqa: F401,F403
