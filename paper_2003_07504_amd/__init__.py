"""MI355X (gfx950) implementation of ILS edge-preserving smoothing
(Liu et al., "Real-time Image Smoothing via Iterative Least Squares").

The compute path is the HIP library libils.so (C ABI in include/ils.h);
this package is its thin Python binding.  Import of the binding is lazy so
that the build step can run without torch's GPU runtime.
"""
__all__ = ["ils"]
