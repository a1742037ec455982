"""The C-ABI library loads and exports every symbol its header declares
(no GPU needed; nothing here launches work)."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "rmips.h")).read()
    return sorted(set(re.findall(r"\b(rmips_[a-z_0-9]+)\s*\(", src)))


def test_header_declarations_match_binding():
    import paper_2504_13445_amd as rm
    assert set(_declared()) == set(rm.EXPORTS)


def test_library_exports_every_symbol():
    import paper_2504_13445_amd as rm
    lib = rm.load()
    for name in _declared():
        assert hasattr(lib, name), name


def test_workspace_queries_validate_sizes():
    import paper_2504_13445_amd as rm
    lib = rm.load()
    assert lib.rmips_thresholds_workspace_size(100, 50, 16, 10, 0) > 0
    assert lib.rmips_thresholds_workspace_size(100, 5, 16, 10, 0) == 0     # k > m
    assert lib.rmips_thresholds_workspace_size(100, 50, 16, 33, 0) == 0    # k > K_MAX
    assert lib.rmips_thresholds_workspace_size(100, 50, 0, 1, 0) == 0      # d = 0
    assert lib.rmips_thresholds_workspace_size(100, 50, 257, 1, 0) == 0    # d > D_MAX
    assert lib.rmips_topn_workspace_size(100, 50, 16, 10, 51, 0) == 0      # N > m
    assert lib.rmips_topn_workspace_size(100, 5000, 16, 10, 1025, 0) == 0  # N > N_MAX
    assert lib.rmips_topn_workspace_size(100, 50, 16, 10, 50, 0) > 0
    assert lib.rmips_scores_workspace_size(100, 7, 16, 0) > 0
    assert lib.rmips_scores_workspace_size(0, 7, 16, 0) == 0
    assert lib.rmips_index_size(100, 50, 16, 25, 0) > 0
    assert lib.rmips_index_workspace_size(100, 50, 16, 25, 1) > 0
    assert lib.rmips_index_size(100, 20, 16, 25, 0) == 0                   # kmax > m
    assert lib.rmips_index_size(100, 50, 16, 33, 0) == 0                   # kmax > K_MAX
    assert lib.rmips_index_workspace_size(100, 50, 16, 0, 2) == 0          # kmax < 1
    assert lib.rmips_budget_index_size(100, 50, 16, 25) > 0
    assert lib.rmips_budget_workspace_size(100, 50, 16, 25, 2) > 0
    assert lib.rmips_budget_index_size(100, 20, 16, 25) == 0               # kmax > m
    assert lib.rmips_budget_workspace_size(100, 50, 16, 33, 0) == 0        # kmax > K_MAX
    assert lib.rmips_budget_workspace_size(100, 50, 16, 10, 7) == 0        # unknown precision


def test_oracle_and_library_share_no_code():
    # the oracle never imports the library and vice versa
    for d, forbidden in (("oracle", "paper_2504_13445_amd"), ("paper_2504_13445_amd", "oracle")):
        for f in os.listdir(os.path.join(ROOT, d)):
            if f.endswith((".py", ".c", ".cpp", ".hip", ".h")):
                txt = open(os.path.join(ROOT, d, f)).read()
                assert not re.search(rf"\bimport\s+{forbidden}\b|\bfrom\s+{forbidden}\b", txt), f
