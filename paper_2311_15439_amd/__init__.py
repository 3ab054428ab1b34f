"""Multiresolution simplex hash encoding for AMD Instinct MI355X (gfx950).

The compute path lives in ``libspx.so`` (hand-written HIP kernels behind a C
ABI, declared in ``include/spx.h``).  ``paper_2311_15439_amd.spx`` is the thin
ctypes binding; importing this package does not load the library.
"""
__all__ = ["spx", "inputs", "torch_ops"]
