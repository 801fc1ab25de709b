"""MI355X-native correlated-sampling phaseless AFQMC walker step.

The compute path is libafqmc.so (hand-written HIP kernels for gfx950 behind
the C ABI of include/afqmc.h); ``paper_1703_01545_amd.afqmc`` is its thin
ctypes binding.  Import the binding explicitly; it raises ImportError when the
library has not been built.
"""
__all__ = ["afqmc", "build"]
