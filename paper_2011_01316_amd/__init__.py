"""MI355X-native exponential-DG hot path (gfx950 HIP kernels behind a C ABI).

The compute path lives in ``libexpdg.so`` (HIP kernels and the C ABI declared
in ``include/expdg.h``); :mod:`paper_2011_01316_amd.binding` is the thin
ctypes layer with the same entry-point names.  Importing this package does not
load the library; :func:`paper_2011_01316_amd.binding.lib` does, and raises if
it has not been built.
"""
__all__ = ["binding", "inputs"]
