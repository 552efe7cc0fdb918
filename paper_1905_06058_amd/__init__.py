"""MI355X-native full-range ISAM operator and MBIR (FISTA) solve.

The computation lives in the HIP library ``libisam.so`` (C ABI in include/isam.h);
this package is its Python binding.
"""
from .isam import (EXPORTS, Batch, FistaInfo, FistaResult, FistaState, Geometry, IsamError, LIB_PATH,  # noqa: F401
                   Plan, direct_static, load_library)

__all__ = ["Plan", "Batch", "Geometry", "IsamError", "FistaResult", "FistaInfo", "FistaState", "load_library",
           "LIB_PATH", "EXPORTS", "direct_static"]
