"""libmm: dense matrix multiplication C = A.B on MI355X (gfx950).

The compute path is libmm.so (HIP kernels behind the C ABI of include/mm.h);
``paper_2408_15384_amd.api`` is its ctypes binding and ``inputs`` the seeded
synthetic input generators.  Importing the package loads nothing; the library
is loaded on first use.
"""
__all__ = ["api", "inputs"]
