"""MI355X-native pair forces with dynamic-size and dynamic-offset cell lists
for deforming periodic boxes (Dobson, Fox & Saracino, arXiv:1412.3784).

The computation lives in the HIP library libnemdcl.so (C ABI in
include/nemdcl.h); `nemdcl` is its ctypes binding.
"""
from . import nemdcl  # noqa: F401  (raises ImportError if the library is not built)
from .nemdcl import Batch, Handle, NclError  # noqa: F401

__all__ = ["nemdcl", "Batch", "Handle", "NclError"]
