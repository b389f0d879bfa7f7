"""MI355X (gfx950) Tucker engine for Matern / Slater covariance tensors.

The compute path is the HIP library libtk.so (C ABI in include/tk.h); `tk` is its ctypes
binding.  Build the library with `python -m paper_1711_06874_amd.build`.
"""
__all__ = ["tk"]
