"""MI355X generalized-stabilizer shot sampler (arXiv 2512.23037 hot path).

The product is libsoft.so (C ABI in include/soft.h, HIP kernels for gfx950);
``paper_2512_23037_amd.soft`` is its ctypes binding.  Importing this package
loads nothing; ``soft.load_library()`` raises if the library is not built.
"""
__all__ = ["soft", "build"]
