"""MI355X-native graph-based S_N transport sweep (Haut et al.).

The compute path lives in the C-ABI library ``libsnsweep.so`` (host setup in
C++, sweep kernels in HIP for gfx950); this package is a thin ctypes binding
with the same function names (``snsw_*``) plus small convenience classes.
PyTorch provides device memory and streams only.
"""
from .binding import (Batch, Context, Net, Problem, SnswError, lib, library_path)  # noqa: F401

__all__ = ["Batch", "Context", "Net", "Problem", "SnswError", "lib", "library_path"]
