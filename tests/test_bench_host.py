"""CPU checks of the bench's static work counts.

The BC7 search fits each distinct 3-subset mask once per mode (Sec. III-B's
exhaustive search over partitions, with recurring subsets shared): the
executed evaluation count the bench reports beside the full count is
re-derived here from the oracle's own 3-subset partition table."""
import os
import re
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def _part3_rows():
    src = open(os.path.join(ROOT, "oracle", "gsbc_oracle.c")).read()
    i = src.index("*P3[64]")
    rows = re.findall(r'"([0-2]{16})"', src[i:src.index("};", i)])
    assert len(rows) == 64
    return rows


def _evals(parts, entries, combos, distinct):
    rows = _part3_rows()
    masks = [sum(1 << t for t in range(16) if rows[p][t] == str(s)) for p in parts for s in range(3)]
    if distinct:
        masks = sorted(set(masks))
    # every member against every entry, initial fit and refit
    return sum(bin(m).count("1") for m in masks) * entries * combos * 2, len(masks)


def test_three_subset_counts():
    full2, n2 = _evals(range(64), 4, 1, False)      # mode 2: 2-bit indices, no p-bits
    full0, n0 = _evals(range(16), 8, 4, False)      # mode 0: 3-bit indices, 4 p-bit pairs
    assert (full2, n2, full0, n0) == (8_192, 192, 16_384, 48)
    assert bench.ALGO_OPS["bc7_search_3subset"] == (full2 + full0) * bench.OPS_PER_EVAL
    ex2, d2 = _evals(range(64), 4, 1, True)
    ex0, d0 = _evals(range(16), 8, 4, True)
    assert (ex2, d2, ex0, d0) == (5_984, 140, 12_288, 36)


def test_executed_evaluations():
    ex2, _ = _evals(range(64), 4, 1, True)
    ex0, _ = _evals(range(16), 8, 4, True)
    two = bench.ALGO_OPS["bc7_search_2subset"] / bench.OPS_PER_EVAL
    one = bench.ALGO_OPS["bc7_search_1subset"] / bench.OPS_PER_EVAL
    assert bench.EXECUTED_EVALS == two + ex2 + ex0 + one
    assert bench.EXECUTED_EVALS * bench.OPS_PER_EVAL < bench.ALGO_OPS["bc7_search_items"]
