"""MI355X-native solve phase of a GNN-smoothed algebraic multigrid pressure solver.

The compute path is libamggnn.so (host Ruge-Stueben setup in C++, HIP kernels for gfx950
behind a C ABI declared in include/amggnn.h). This package holds its ctypes binding
(``capi``, same names as the C functions) and the torch-memory plumbing (``solver``).
The library is loaded on first use (``capi.lib()``) and raises if it has not been built;
there is no other implementation to fall back to.
"""
from . import capi
from .capi import AmggError

__all__ = ["capi", "AmggError"]
