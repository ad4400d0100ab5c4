"""Dynamic-data-rate actor networks on AMD MI355X (gfx950).

The compute path is libdfhip.so (HIP kernels behind the C ABI declared in
include/dfhip.h).  ``dfhip`` is the thin ctypes binding (same names as the C
entry points), ``graph`` a convenience wrapper for building networks,
``autograd`` the torch.autograd functions for coefficient adaptation and
``tune`` the tile autotuner.  Importing ``dfhip`` fails if the library is
not built: there is no fallback path.
"""
__all__ = ["dfhip", "graph", "autograd", "tune"]
