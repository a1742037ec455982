"""librmips: exact reverse k-MIPS top-N on AMD Instinct MI355X (gfx950).

Python side of the C ABI in include/rmips.h; see _lib for the calls.
"""
from ._lib import (EXPORTS, K_MAX, N_MAX, D_MAX, BudgetIndex, Index, RmipsError, SoftScore,
                   load, profile, scores, set_profiling, soft_bwd, soft_fwd, soft_fwd_grad,
                   soft_scale, sync, thresholds, topn, topn_workspace)

__all__ = ["EXPORTS", "K_MAX", "N_MAX", "D_MAX", "BudgetIndex", "Index", "RmipsError",
           "SoftScore", "load", "profile", "scores", "set_profiling", "soft_bwd", "soft_fwd",
           "soft_fwd_grad", "soft_scale", "sync", "thresholds", "topn", "topn_workspace"]
