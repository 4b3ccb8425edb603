"""MI355X-native multi-spin-coded checkerboard Metropolis sweep of the 2D Ising model.

The compute path is libising.so (HIP for gfx950, C ABI in include/ising.h);
``paper_1007_3726_amd.ising`` is its ctypes binding.  Importing this package
does not touch the GPU.
"""
__all__ = ["ising", "build"]
