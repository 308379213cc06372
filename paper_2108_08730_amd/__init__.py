"""helm27: wavelength-adaptive 27-point frequency-domain Helmholtz on MI355X.

The compute path lives in libhelm27.so (C ABI in include/helm27.h, HIP kernels
for gfx950); this package is a marshalling layer over it.  Importing
``paper_2108_08730_amd.api`` fails loudly when the library is not built.
"""
__all__ = ["api", "build"]
