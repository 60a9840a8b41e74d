"""MI355X-native isospectral-midpoint Zeitlin--Euler step on the sphere (arXiv 2206.05466).

The computation lives in ``libzeuler.so`` (HIP, gfx950; C ABI in ``include/zeuler.h``);
``zeuler`` is its ctypes binding.
"""

from .zeuler import (
    LIB_PATH, PREC_CRT, PREC_FP64, PREC_MIXED, PREC_SPLIT, SIGNATURES, Ensemble, StepInfo, Zeuler, ZeulerError,
    load_library, zgemm_noalloc,
)

__all__ = ["LIB_PATH", "PREC_CRT", "PREC_FP64", "PREC_MIXED", "PREC_SPLIT", "SIGNATURES", "Ensemble", "StepInfo", "Zeuler",
           "ZeulerError", "load_library", "zgemm_noalloc"]
