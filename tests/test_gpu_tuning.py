"""The autotuned defaults reach the traversal: g5_build_csr picks the table
entry tuned at the scale nearest to ceil(log2 n) (the first of two equally
near), a traversal reports that entry's alpha, beta, lane-scan width and
bottom-up grid, and explicit parameters override it.  The tuning depends on n
only, so each graph is a short path in a vertex range of the given scale."""
import os
import re

import numpy as np
import pytest

import paper_2012_13548_amd as g5
from tests.gpu_util import to_dev

pytestmark = pytest.mark.gpu

ROW = re.compile(r"^\{(\d+), ([\d.]+), ([\d.]+), (\d+), (\d+), ([12]), ([01]), (\d+), "
                 r"([\d.]+), ([\d.]+), (\d+), (-?[\d.]+)\},$")


def shipped_table():
    here = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    text = open(os.path.join(here, "paper_2012_13548_amd", "csrc", "tuned_table.inc")).read()
    out = []
    for line in text.splitlines():
        m = ROW.match(line)
        if m:
            g = m.groups()
            out.append(dict(scale=int(g[0]), alpha=float(g[1]), beta=float(g[2]),
                            lane_scan=int(g[3]), blocks_per_cu=int(g[4])))
    return out


def nearest(table, scale):
    best = table[0]
    for t in table:
        if abs(t["scale"] - scale) < abs(best["scale"] - scale):
            best = t
    return best


@pytest.mark.parametrize("scale", [10, 21, 23, 24, 26])
def test_tuned_defaults_applied(scale):
    table = shipped_table()
    assert len(table) >= 2
    want = nearest(table, scale)
    n = 1 << scale
    path = np.array([[0, 1], [1, 2], [2, 3], [3, n - 1]], dtype=np.int64)
    csr = g5.build_csr(to_dev(path), n)
    _, level, st = g5.bfs(csr, 0, stats=True)
    lv = level.cpu().numpy()
    assert lv[[0, 1, 2, 3, n - 1]].tolist() == [0, 1, 2, 3, 4] and (lv >= 0).sum() == 5
    assert st["alpha"] == pytest.approx(want["alpha"]) and st["beta"] == pytest.approx(want["beta"])
    assert st["lane_scan"] == want["lane_scan"] and st["blocks_per_cu"] == want["blocks_per_cu"]
    _, _, st2 = g5.bfs(csr, 0, stats=True, alpha=3.5, beta=5.5, lane_scan=2, blocks_per_cu=7)
    assert (st2["alpha"], st2["beta"], st2["lane_scan"], st2["blocks_per_cu"]) == (3.5, 5.5, 2, 7)
