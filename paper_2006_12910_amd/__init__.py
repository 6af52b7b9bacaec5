"""MI355X (gfx950) D2Q9 lattice-Boltzmann hot path of arXiv:2006.12910.

The computation lives in the HIP library liblb.so (C ABI in include/lb.h);
this package holds its sources (csrc/), the build script and a thin ctypes
binding (lb.py).  Importing the binding needs the built library.
"""
__all__ = ["lb", "build", "inputs"]
