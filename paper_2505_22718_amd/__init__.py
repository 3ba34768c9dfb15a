"""MI355X (gfx950) beyond-Limber angular power spectra: FFTLog k-windows and their projection.

The compute path is libswiftcl.so (hand-written HIP, include/swiftcl.h).  This package holds
the ctypes binding (binding.py), a torch-facing Plan (plan.py) and the autograd Function
(autograd.py).  PyTorch provides device memory and streams only.
"""
from .binding import (SWIFTCL_CLUSTERING, SWIFTCL_FP32, SWIFTCL_FP64, SWIFTCL_LENSING,  # noqa: F401
                      SWIFTCL_SPLIT_BF16, SwiftclError)

__all__ = ["SwiftclError", "SWIFTCL_CLUSTERING", "SWIFTCL_LENSING", "SWIFTCL_FP64", "SWIFTCL_FP32",
           "SWIFTCL_SPLIT_BF16"]
