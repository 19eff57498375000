"""MI355X-native block one-sided Jacobi SVD and hyperbolic SVD in FP64.

The computation runs in the HIP library ``_lib/libjsvd.so`` (C ABI in
``include/jsvd.h``); this package is its Python binding.  See
``_binding`` for the calls.
"""
from ._binding import (EXPORTS, Batch, JsvdError, STRATEGIES, batched_block_min_n,  # noqa: F401
                       colnorms, diag_fp64, diag_refined, rdssq_bounds, gesvd, gesvd_batched, gesvd_full, hsvd, lib,
                       reserve_batched, strategy_order, strategy_table, svd_backward,
                       workspace_size, workspace_size_batched)
from .autograd import JacobiSVD, svd  # noqa: F401,E402

__all__ = ["gesvd", "gesvd_full", "hsvd", "gesvd_batched", "Batch", "svd", "JacobiSVD", "svd_backward", "strategy_table", "strategy_order", "diag_fp64", "diag_refined", "colnorms", "rdssq_bounds", "lib", "JsvdError", "batched_block_min_n",
           "workspace_size", "workspace_size_batched", "reserve_batched"]
