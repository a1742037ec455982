"""librmips: exact reverse k-MIPS top-N on AMD Instinct MI355X (gfx950).

Python side of the C ABI in include/rmips.h; see _lib for the calls.
"""
from ._lib import (EXPORTS, K_MAX, N_MAX, D_MAX, RmipsError, SoftScore, load,
                   scores, soft_bwd, soft_fwd, thresholds, topn, topn_workspace)

__all__ = ["EXPORTS", "K_MAX", "N_MAX", "D_MAX", "RmipsError", "SoftScore", "load",
           "scores", "soft_bwd", "soft_fwd", "thresholds", "topn", "topn_workspace"]
