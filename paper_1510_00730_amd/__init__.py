"""MI355X-native multideterminant wavefunction evaluator (arXiv:1510.00730).

The hot path lives in libmdet.so (HIP kernels for gfx950 behind the C ABI of
include/mdet.h); this package is its Python binding.
"""
from .binding import (MDET_FP64, MDET_MIXED, METHOD_SM_CHAIN, METHOD_TABLE,  # noqa: F401
                      W_FALLBACK, W_NODE, W_OK, Evaluator, MdetError, load_library,
                      norm_truncation)

__all__ = ["Evaluator", "MdetError", "MDET_FP64", "MDET_MIXED", "W_OK", "W_FALLBACK", "W_NODE",
           "METHOD_TABLE", "METHOD_SM_CHAIN", "load_library", "norm_truncation"]
