"""MI355X-native CRKSPH neighbour passes (Frontiere et al., CRK-HACC, Sec. 2.2, 3.6).

Python face of ``libcrk.so``: each method of :class:`Context` marshals torch
device tensors into one C-ABI call of the same name (``include/crk.h``); all
arithmetic runs in the library's HIP kernels. Importing this package never
falls back to anything else: if the library is missing or no GPU is present,
the calls raise.
"""
from ._lib import (CRK_FP64, CRK_MIXED, CRK_MIXED_ADAPT, CrkError, Context, Params, lib, library_path,
                   version)

__all__ = ["CRK_FP64", "CRK_MIXED", "CRK_MIXED_ADAPT", "CrkError", "Context", "Params", "lib", "library_path",
           "version"]
