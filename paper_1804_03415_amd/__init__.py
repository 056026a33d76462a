"""Hierarchically preconditioned eigensolver on MI355X (HIP / CDNA4).

The compute path is the C-ABI library libmmdeig.so (include/mmdeig.h); this
package only marshals arguments to it.
"""
from ._lib import MMDError, lib  # noqa: F401
from .api import (Decomposition, EigLeftmost, build_options, eig_leftmost_batched,  # noqa: F401
                  gemm, gram, solver_options, spmm, spmm_noalloc)

__all__ = ["Decomposition", "EigLeftmost", "MMDError", "build_options", "eig_leftmost_batched",
           "solver_options", "spmm", "spmm_noalloc", "gram", "gemm", "lib"]
