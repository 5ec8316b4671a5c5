"""MI355X (gfx950) hot path of compressive spectral clustering.

The work is done by libcsc.so (hand-written HIP, C ABI in include/csc.h);
``api`` marshals arguments from PyTorch tensors.  Importing the package does
not load the library; the first call does, and fails if it was not built.
"""
from ._lib import CscError, LIB_PATH  # noqa: F401

__all__ = ["api", "CscError", "LIB_PATH"]
