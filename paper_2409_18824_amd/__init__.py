"""MI355X-native 3D 7-point Jacobi / Poisson library with Fortran array semantics.

The compute lives in ``libj3d.so`` (HIP kernels for gfx950 behind a C ABI,
declared in ``include/j3d.h``); ``paper_2409_18824_amd.j3d`` is its ctypes
binding.  Importing the package does not load the library; importing
``paper_2409_18824_amd.j3d`` does, and fails if it has not been built.
"""

__all__ = ["j3d"]
