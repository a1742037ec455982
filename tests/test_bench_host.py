"""Host logic of bench.py (no GPU): the per-launch work that the per-kernel
table divides by each kernel's time, with and without the rotated pre-pass
of the Eq. 3 bound."""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import bench  # noqa: E402


def _stats(prepass, rebound_items, rebound_pairs):
    return [{"thresh_pairs": 1.0e9, "refine_pairs": 0.0, "count_pairs": 5.0e8,
             "bound_pairs": 6.0e9, "rebound_pairs": rebound_pairs,
             "prepass_dprime": prepass, "rebound_items": rebound_items,
             "cand_listed": 1.0e6}]


def test_bound_work_with_prepass():
    n, m, d = 20000, 3000, 200
    prof = [("k_bound", 1, 8.0), ("k_bound/rebound", 1, 4.0), ("k_aug_ident", 2, 1.0)]
    t = bench.kernel_table(prof, _stats(62, 500, 2.0e9), 1, n, m, d, 10, "fp32")
    # the pre-pass: d' + 2 = 64 terms per pair; the second bound: d + 2
    assert t["k_bound"]["work_per_launch"] == 2.0 * 64 * 6.0e9
    assert t["k_bound/rebound"]["work_per_launch"] == 2.0 * 202 * 2.0e9
    # identity rows: every user and the 500 re-bounded items, 224 BF16
    # values written per row (d + 2 rounded up to 32 past 176 terms)
    rows = n + 500
    assert t["k_aug_ident"]["work_per_launch"] == (rows * 4.0 * d + rows * 2.0 * 224) / 2
    assert abs(t["k_bound"]["achieved"] - 2.0 * 64 * 6.0e9 / 8.0e-3 / 1e12) < 1e-9


def test_bound_work_without_prepass():
    n, m, d = 20000, 3000, 100
    prof = [("k_bound", 1, 8.0), ("k_aug_ident", 2, 1.0)]
    t = bench.kernel_table(prof, _stats(0, 0, 0.0), 1, n, m, d, 10, "bf16")
    assert t["k_bound"]["work_per_launch"] == 2.0 * 102 * 6.0e9
    mpad = (m + 63) // 64 * 64
    assert t["k_aug_ident"]["work_per_launch"] == ((n + m) * 4.0 * d + (n + mpad) * 2.0 * 112) / 2
    assert "k_bound/rebound" not in t
