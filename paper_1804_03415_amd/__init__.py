"""Hierarchically preconditioned eigensolver on MI355X (HIP / CDNA4).

The compute path is the C-ABI library libmmdeig.so (include/mmdeig.h); this
package only marshals arguments to it.
"""
from ._lib import MMDError, lib  # noqa: F401
from .api import Decomposition, EigLeftmost, build_options, solver_options, spmm  # noqa: F401

__all__ = ["Decomposition", "EigLeftmost", "MMDError", "build_options", "solver_options",
           "spmm", "lib"]
