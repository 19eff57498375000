"""MI355X-native block one-sided Jacobi SVD and hyperbolic SVD in FP64.

The computation runs in the HIP library ``_lib/libjsvd.so`` (C ABI in
``include/jsvd.h``); this package is its Python binding.  See
``_binding`` for the calls.
"""
from ._binding import (EXPORTS, JsvdError, STRATEGIES, diag_fp64, gesvd, hsvd, lib,  # noqa: F401
                       strategy_order, strategy_table)

__all__ = ["gesvd", "hsvd", "strategy_table", "strategy_order", "diag_fp64", "lib", "JsvdError"]
