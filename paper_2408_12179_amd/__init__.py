"""MI355X-native HPR-LP: the HPR iteration for linear programming on gfx950.

The solver lives in ``libhprlp.so`` (C ABI in ``include/hprlp.h``); ``hprlp`` is its thin
Python binding.
"""
from .hprlp import (FP64, FP64_A32, MIXED, HPRLPError, Solution, Solver, default_options, load,
                    workspace_bytes, workspace_bytes_batched)

__all__ = ["FP64", "FP64_A32", "MIXED", "HPRLPError", "Solution", "Solver", "default_options", "load",
           "workspace_bytes", "workspace_bytes_batched"]
