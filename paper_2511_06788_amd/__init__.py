"""MI355X (gfx950) implementation of the orthogonality-preserving eigensolver step.

The computation lives in the HIP library ``libope.so`` (sources in ``csrc/``,
C ABI in ``include/ope.h``); :mod:`paper_2511_06788_amd.ope` is its ctypes
binding and :mod:`paper_2511_06788_amd.build` compiles it for gfx950.
"""
__all__ = ["ope", "build"]
