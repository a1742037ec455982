"""Seeded synthetic inputs shared by the oracle and the GPU path.

This module only draws random numbers; it holds none of the method's
arithmetic (no inner products, no top-k, no counting).
"""
from .generate import (CONFIGS, Config, isotropic, clustered, make_config,
                       make_queries, subsample_users)

__all__ = ["CONFIGS", "Config", "isotropic", "clustered", "make_config",
           "make_queries", "subsample_users"]
