"""MI355X-native randomized column-pivoted QR (Duersch & Gu, arXiv:2008.04447).

The computation lives in ``librqrcp.so`` (HIP kernels for gfx950 behind the C ABI
of ``include/rqrcp.h``); this package only marshals torch tensors into it.
Importing the package does not load the library; the first call does, and it
raises if the library has not been built.
"""
from ._lib import (LIB_PATH, RQ_E_DEVICE, RQ_E_HIP, RQ_E_NOMEM, RQ_E_UNSUPPORTED, RQ_FP64,
                   RQ_MIXED_BF16, RQ_OK, SIGNATURES, RQError, load)

__all__ = ["LIB_PATH", "SIGNATURES", "RQError", "load", "RQ_OK", "RQ_E_HIP", "RQ_E_NOMEM",
           "RQ_E_UNSUPPORTED", "RQ_E_DEVICE", "RQ_FP64", "RQ_MIXED_BF16"]
