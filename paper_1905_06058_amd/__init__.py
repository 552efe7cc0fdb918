"""MI355X-native full-range ISAM operator and MBIR (FISTA) solve.

The computation lives in the HIP library ``libisam.so`` (C ABI in include/isam.h);
this package is its Python binding.
"""
from .isam import (EXPORTS, Batch, FistaInfo, FistaResult, Geometry, IsamError, LIB_PATH, Plan,  # noqa: F401
                   load_library)

__all__ = ["Plan", "Batch", "Geometry", "IsamError", "FistaResult", "FistaInfo", "load_library", "LIB_PATH",
           "EXPORTS"]
