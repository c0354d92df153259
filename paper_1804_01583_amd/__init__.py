"""MI355X-native projected Krylov simulation for affine-system verification
(Bak, Tran, Johnson, arXiv 1804.01583).

The computation lives in libkry.so (HIP kernels for gfx950 behind the C ABI
of include/kry.h); ``paper_1804_01583_amd.kry`` is its ctypes binding.
Importing the binding fails when the library has not been built.
"""
__all__ = ["kry"]
