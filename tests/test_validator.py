"""The validators reject broken BFS trees (mutation tests).

Each mutation breaks one rule of a valid result; both the CSR validator and the
tuple-list validator must reject it.
"""
import numpy as np
import pytest

import kronecker as K
import oracle as O
from tests import graphs as G


@pytest.fixture(scope="module")
def case():
    scale = 11
    n = 1 << scale
    e = K.edges_host(scale)
    csr = O.build_csr(e, n)
    root = K.select_roots(K.nonisolated_host(e, n), 1, K.root_seed(scale))[0]
    parent, level = O.bfs(csr, root)
    label = O.components(e, n)
    return e, n, csr, root, parent, level, label


def both(case, parent, level):
    e, n, csr, root, _, _, label = case
    return (O.validate(csr, root, parent, level, label),
            O.validate_edges(e, n, root, parent, level))


def test_valid(case):
    _, _, _, _, parent, level, _ = case
    assert both(case, parent, level) == (0, 0)


def pick(level, lv):
    return int(np.flatnonzero(level == lv)[0])


def test_root_not_own_parent(case):
    _, _, _, root, parent, level, _ = case
    p = parent.copy()
    p[root] = pick(level, 1)
    assert all(r != 0 for r in both(case, p, level))


def test_parent_not_a_neighbour(case):
    e, n, csr, root, parent, level, _ = case
    # a vertex at level 3 given a level-2 parent that is not adjacent to it
    v = pick(level, 3)
    adj = set(csr.row(v).tolist())
    cand = [u for u in np.flatnonzero(level == 2) if u not in adj]
    p = parent.copy()
    p[v] = cand[0]
    assert both(case, p, level) == (3, 3)


def test_parent_same_level(case):
    _, _, csr, _, parent, level, _ = case
    v = next(v for v in np.flatnonzero(level == 2)
             if any(level[u] == 2 for u in csr.row(v)))
    u = next(u for u in csr.row(v) if level[u] == 2)
    p = parent.copy()
    p[v] = u
    assert both(case, p, level) == (4, 4)


def test_level_off_by_one(case):
    _, _, _, _, parent, level, _ = case
    l2 = level.copy()
    l2[pick(level, 2)] = 3
    assert all(r != 0 for r in both(case, parent, l2))


def test_missing_reached_vertex(case):
    _, _, _, _, parent, level, _ = case
    v = int(np.flatnonzero(level == level.max())[0])
    p, l2 = parent.copy(), level.copy()
    p[v] = -1
    l2[v] = -1
    assert both(case, p, l2) == (5, 5)


def test_extra_reached_vertex(case):
    _, _, _, _, parent, level, label = case
    v = int(np.flatnonzero(level < 0)[0])
    p, l2 = parent.copy(), level.copy()
    p[v] = v
    l2[v] = 1
    r = both(case, p, l2)
    assert r[0] != 0 and r[1] != 0


def test_parent_without_level(case):
    _, _, _, _, parent, level, _ = case
    v = int(np.flatnonzero(level < 0)[0])
    p = parent.copy()
    p[v] = 0
    assert both(case, p, level) == (2, 2)


def test_second_level_zero(case):
    e, n, csr, root, parent, level, _ = case
    v = pick(level, 1)
    l2 = level.copy()
    l2[v] = 0
    p = parent.copy()
    p[v] = v
    assert all(r != 0 for r in both(case, p, l2))


def test_shortcut_levels_rejected():
    # levels consistent with a valid-looking parent chain but not shortest:
    # on a cycle, walking the long way round breaks the edge rule (6).
    e, n = G.cycle(8)
    csr = O.build_csr(e, n)
    label = O.components(e, n)
    level = np.array([0, 1, 2, 3, 4, 5, 6, 7], np.int32)
    parent = np.array([0, 0, 1, 2, 3, 4, 5, 6], np.int32)
    assert O.validate(csr, 0, parent, level, label) == 6
    assert O.validate_edges(e, n, 0, parent, level) == 6


# check_parents: the parent rules alone, for level arrays already compared with
# the oracle's.  Each parent mutation above is rejected with the same rule as
# the full CSR validator, and random parent mutations agree with it on
# accept/reject.

def test_check_parents_valid(case):
    _, _, csr, root, parent, level, _ = case
    assert O.check_parents(csr, root, parent, level) == 0
    assert O.check_parents(csr, root, O.min_parents(csr, root, level), level) == 0


def test_check_parents_rules(case):
    e, n, csr, root, parent, level, label = case
    p = parent.copy()
    p[root] = pick(level, 1)
    assert O.check_parents(csr, root, p, level) == 1
    v = pick(level, 3)
    adj = set(csr.row(v).tolist())
    p = parent.copy()
    p[v] = [u for u in np.flatnonzero(level == 2) if u not in adj][0]
    assert O.check_parents(csr, root, p, level) == 3
    v = next(v for v in np.flatnonzero(level == 2) if any(level[u] == 2 for u in csr.row(v)))
    p = parent.copy()
    p[v] = next(u for u in csr.row(v) if level[u] == 2)
    assert O.check_parents(csr, root, p, level) == 4
    p = parent.copy()
    p[int(np.flatnonzero(level < 0)[0])] = 0
    assert O.check_parents(csr, root, p, level) == 2
    p = parent.copy()
    p[pick(level, 2)] = -1
    assert O.check_parents(csr, root, p, level) == 2


def test_check_parents_agrees_with_validate(case):
    _, n, csr, root, parent, level, label = case
    rng = np.random.default_rng(5)
    reached = np.flatnonzero((level > 0))
    for _ in range(300):
        p = parent.copy()
        v = int(rng.choice(reached))
        p[v] = int(rng.choice(csr.row(v))) if rng.random() < 0.7 else int(rng.integers(0, n))
        full = O.validate(csr, root, p, level, label)
        assert (O.check_parents(csr, root, p, level) == 0) == (full == 0), (v, p[v], full)
