"""Pins for the CPU oracle (oracle/), each against something other than itself.

* Closed forms for hop distance on paths, stars, grids, cycles, complete graphs,
  complete binary trees and disjoint unions.
* Brute force: every labelled simple graph on 5 vertices from every root
  against Floyd-Warshall, and random graphs on up to 64 vertices against
  boolean powers of (A + I).
* Library special case: scipy.sparse.csgraph.shortest_path(unweighted=True)
  on Kronecker graphs, scipy's connected_components for the union-find, and
  scipy's COO->CSR with duplicates summed for the CSR.
* The hand-worked fixtures in tests/golden/ (CSR empty-row rule of Section 2.2,
  level-synchronisation example of Section 2.3.2).
"""
import itertools

import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse import csgraph

import kronecker as K
import oracle as O
from tests import graphs as G
from tests import golden


def run(edges, n, root):
    csr = O.build_csr(edges, n)
    parent, level = O.bfs(csr, root)
    label = O.components(edges, n)
    assert O.validate(csr, root, parent, level, label) == 0
    assert O.validate_edges(edges, n, root, parent, level) == 0
    return csr, parent, level


def dist_to_level(d):
    d = np.asarray(d, dtype=np.float64)
    return np.where(np.isinf(d), -1, d).astype(np.int64)


# --------------------------------------------------------------- closed forms
@pytest.mark.parametrize("n,r", [(1, 0), (2, 1), (10, 0), (10, 9), (33, 17)])
def test_path(n, r):
    e, n = G.path(n)
    if e.size == 0:
        e = np.zeros((0, 2), np.int64)
    _, parent, level = run(e, n, r)
    assert np.array_equal(level, G.path_dist(n, r))


@pytest.mark.parametrize("leaves,r", [(1, 0), (7, 0), (7, 3), (300, 0), (300, 299)])
def test_star(leaves, r):
    e, n = G.star(leaves)
    _, parent, level = run(e, n, r)
    assert np.array_equal(level, G.star_dist(leaves, r))
    if r == 0:
        assert np.all(parent[1:] == 0)


@pytest.mark.parametrize("path_len,leaves", [(1, 3), (5, 1), (300, 40)])
def test_broom(path_len, leaves):
    e, n = G.broom(path_len, leaves)
    _, parent, level = run(e, n, 0)
    assert np.array_equal(level, G.broom_dist(path_len, leaves))
    # a pendant's only neighbour is its leaf
    assert np.array_equal(parent[path_len + leaves:], np.arange(path_len, path_len + leaves))


@pytest.mark.parametrize("a,b,r", [(1, 5, 2), (4, 4, 0), (7, 3, 10), (20, 31, 311)])
def test_grid(a, b, r):
    e, n = G.grid(a, b)
    _, _, level = run(e, n, r)
    assert np.array_equal(level, G.grid_dist(a, b, r))


@pytest.mark.parametrize("n,r", [(3, 0), (4, 2), (9, 4), (64, 5)])
def test_cycle(n, r):
    e, n = G.cycle(n)
    _, _, level = run(e, n, r)
    assert np.array_equal(level, G.cycle_dist(n, r))


@pytest.mark.parametrize("n", [2, 5, 17])
def test_complete(n):
    e, n = G.complete(n)
    for r in (0, n - 1):
        _, parent, level = run(e, n, r)
        assert np.array_equal(level, G.complete_dist(n, r))
        assert np.all(parent[np.arange(n) != r] == r)


@pytest.mark.parametrize("depth,r", [(1, 0), (4, 0), (4, 9), (6, 100)])
def test_binary_tree(depth, r):
    e, n = G.binary_tree(depth)
    _, parent, level = run(e, n, r)
    assert np.array_equal(level, G.binary_tree_dist(n, r))


def test_disjoint_union_and_isolated():
    e, n, offs = G.disjoint_union(G.path(5), G.cycle(6), G.star(4))
    n += 3  # three isolated vertices at the end
    _, parent, level = run(e, n, offs[1] + 2)
    expect = np.full(n, -1)
    expect[offs[1]:offs[1] + 6] = G.cycle_dist(6, 2)
    assert np.array_equal(level, expect)
    assert np.all(parent[expect < 0] == -1)


def test_isolated_root():
    e = np.array([[1, 2]], np.int64)
    _, parent, level = run(e, 4, 0)
    assert level.tolist() == [0, -1, -1, -1]
    assert parent.tolist() == [0, -1, -1, -1]


# --------------------------------------------------------------- brute force
def floyd_warshall(n, pairs):
    INF = 10 ** 6
    d = np.full((n, n), INF, dtype=np.int64)
    np.fill_diagonal(d, 0)
    for u, v in pairs:
        d[u, v] = d[v, u] = 1
    for k in range(n):
        d = np.minimum(d, d[:, k:k + 1] + d[k:k + 1, :])
    return np.where(d >= INF, -1, d)


def test_exhaustive_five_vertex_graphs():
    n = 5
    all_pairs = list(itertools.combinations(range(n), 2))
    for mask in range(1 << len(all_pairs)):
        pairs = [p for i, p in enumerate(all_pairs) if mask >> i & 1]
        e = G.as_edges(pairs) if pairs else np.zeros((0, 2), np.int64)
        fw = floyd_warshall(n, pairs)
        csr = O.build_csr(e, n)
        label = O.components(e, n)
        for r in range(n):
            parent, level = O.bfs(csr, r)
            assert np.array_equal(level, fw[r]), (pairs, r)
            assert O.validate(csr, r, parent, level, label) == 0


def matrix_power_levels(n, pairs, r):
    """Smallest k with ((A + I)^k)[r, v] != 0, by repeated boolean products."""
    a = np.eye(n, dtype=bool)
    for u, v in pairs:
        a[u, v] = a[v, u] = True
    lev = np.full(n, -1)
    reach = np.zeros(n, dtype=bool)
    reach[r] = True
    lev[r] = 0
    for k in range(1, n):
        nxt = (reach.astype(np.int64) @ a.astype(np.int64)) > 0
        lev[nxt & (lev < 0)] = k
        reach = nxt
    return lev


def test_random_graphs_vs_matrix_powers():
    rng = np.random.default_rng(7)
    for trial in range(60):
        n = int(rng.integers(2, 65))
        p = float(rng.choice([0.02, 0.05, 0.1, 0.3]))
        e, n = G.random_graph(rng, n, p)
        csr = O.build_csr(e, n) if e.size else O.build_csr(np.zeros((0, 2), np.int64), n)
        for r in rng.integers(0, n, size=3):
            _, level = O.bfs(csr, int(r))
            assert np.array_equal(level, matrix_power_levels(n, e.tolist(), int(r)))


# --------------------------------------------------------------- library cases
def scipy_csr(edges, n):
    e = edges[edges[:, 0] != edges[:, 1]]
    rows = np.concatenate([e[:, 0], e[:, 1]])
    cols = np.concatenate([e[:, 1], e[:, 0]])
    a = sp.coo_matrix((np.ones(rows.size), (rows, cols)), shape=(n, n)).tocsr()
    a.sum_duplicates()
    a.sort_indices()
    return a


@pytest.mark.parametrize("scale", [8, 10, 12, 14])
def test_csr_vs_scipy(scale):
    n = 1 << scale
    e = K.edges_host(scale)
    csr = O.build_csr(e, n)
    a = scipy_csr(e, n)
    assert np.array_equal(csr.row_ptr, a.indptr.astype(np.int64))
    assert np.array_equal(csr.col_idx, a.indices.astype(np.int32))
    # invariants of the layout
    assert csr.row_ptr[0] == 0 and csr.row_ptr[-1] == csr.nnz
    assert np.all(np.diff(csr.row_ptr) >= 0)
    rows = np.repeat(np.arange(n), np.diff(csr.row_ptr))
    assert np.all(rows != csr.col_idx)
    s = rows.astype(np.int64) * n + csr.col_idx
    assert np.all(np.diff(s) > 0)          # rows strictly ascending, unique
    t = np.sort(csr.col_idx.astype(np.int64) * n + rows)
    assert np.array_equal(s, t)            # symmetric


@pytest.mark.parametrize("scale,nroots", [(10, 8), (12, 6), (14, 4)])
def test_kronecker_vs_scipy_shortest_path(scale, nroots):
    n = 1 << scale
    e = K.edges_host(scale)
    csr = O.build_csr(e, n)
    roots = K.select_roots(K.nonisolated_host(e, n), nroots, K.root_seed(scale))
    a = scipy_csr(e, n)
    d = csgraph.shortest_path(a, directed=False, unweighted=True, indices=roots)
    label = O.components(e, n)
    for i, r in enumerate(roots):
        parent, level = O.bfs(csr, r)
        assert np.array_equal(level, dist_to_level(d[i]))
        assert O.validate(csr, r, parent, level, label) == 0


@pytest.mark.parametrize("scale", [10, 13])
def test_components_vs_scipy(scale):
    n = 1 << scale
    e = K.edges_host(scale)
    label = O.components(e, n)
    ncomp, lab2 = csgraph.connected_components(scipy_csr(e, n), directed=False)
    assert len(np.unique(label)) == ncomp
    # same partition: the map label -> lab2 is a bijection
    pairs = np.unique(np.stack([label, lab2], 1), axis=0)
    assert pairs.shape[0] == ncomp


# --------------------------------------------------------------- fixtures
def test_golden_csr_empty_rows():
    g = golden.load("csr_empty_rows.txt")
    csr = O.build_csr(g["edges"], g["n"])
    assert csr.row_ptr.tolist() == g["row_ptr"].tolist()
    assert csr.col_idx.tolist() == g["col_idx"].tolist()


@pytest.mark.parametrize("name", ["fail1.txt", "two_components.txt"])
def test_golden_levels(name):
    g = golden.load(name)
    _, parent, level = run(g["edges"], g["n"], g["root"])
    for v, l in g["level"].items():
        assert level[v] == l, (v, level[v], l)
    for v, ch in g["parent_choices"].items():
        assert parent[v] in ch


def test_multigraph_same_as_simple():
    # repeated tuples and self-loops never change distances (Section 2.1)
    e, n = G.grid(6, 7)
    noisy = np.concatenate([e, e[::-1], e[:, ::-1], np.stack([np.arange(n)] * 2, 1)])
    c1, _, l1 = run(e, n, 5)
    c2, _, l2 = run(noisy, n, 5)
    assert np.array_equal(l1, l2)
    assert np.array_equal(c1.row_ptr, c2.row_ptr)
    assert np.array_equal(c1.col_idx, c2.col_idx)


# --------------------------------------------------------------- TEPS count
def test_teps_edges_closed_forms():
    e, n = G.star(9)
    csr, _, level = run(e, n, 3)
    assert O.teps_edges(csr, level) == 9
    e, n = G.complete(8)
    csr, _, level = run(e, n, 0)
    assert O.teps_edges(csr, level) == 28
    e, n, offs = G.disjoint_union(G.complete(5), G.path(10))
    noisy = np.concatenate([e, e, [[0, 0]]])
    csr, _, level = run(noisy, n, offs[1])
    assert O.teps_edges(csr, level) == 9
    csr, _, level = run(noisy, n, 0)
    assert O.teps_edges(csr, level) == 10


# --------------------------------------------------------------- batch, errors
def test_batch_matches_single():
    scale = 10
    n = 1 << scale
    e = K.edges_host(scale)
    csr = O.build_csr(e, n)
    roots = K.select_roots(K.nonisolated_host(e, n), 8, K.root_seed(scale))
    parents, levels = O.bfs_batch(csr, roots + [roots[0]])
    assert levels.dtype == np.int8 and levels.shape == (9, n)
    for i, r in enumerate(roots + [roots[0]]):
        p, l = O.bfs(csr, r)
        assert np.array_equal(levels[i].astype(np.int32), l)
        assert np.array_equal(parents[i], p)


def test_errors():
    with pytest.raises(ValueError):
        O.build_csr(np.array([[0, 5]]), 5)
    with pytest.raises(ValueError):
        O.build_csr(np.array([[-1, 2]]), 5)
    csr = O.build_csr(np.array([[0, 1]]), 3)
    with pytest.raises(ValueError):
        O.bfs(csr, 3)
    with pytest.raises(ValueError):
        O.bfs(csr, -1)


def test_empty_edge_list():
    csr = O.build_csr(np.zeros((0, 2), np.int64), 4)
    assert csr.row_ptr.tolist() == [0, 0, 0, 0, 0] and csr.nnz == 0
    parent, level = O.bfs(csr, 2)
    assert level.tolist() == [-1, -1, 0, -1]


# --------------------------------------------------------------- min parents
def test_min_parents_closed_forms():
    e, n = G.path(12)
    csr, _, level = run(e, n, 4)
    p = O.min_parents(csr, 4, level)
    expect = np.array([1, 2, 3, 4, 4, 4, 5, 6, 7, 8, 9, 10])
    assert np.array_equal(p, expect)
    e, n = G.binary_tree(5)
    csr, _, level = run(e, n, 0)
    p = O.min_parents(csr, 0, level)
    assert p[0] == 0 and np.array_equal(p[1:], (np.arange(1, n) - 1) // 2)
    a, b = 6, 9
    e, n = G.grid(a, b)
    csr, _, level = run(e, n, 0)
    p = O.min_parents(csr, 0, level)
    i, j = np.divmod(np.arange(n), b)
    expect = np.where(i > 0, (i - 1) * b + j, i * b + j - 1)
    expect[0] = 0
    assert np.array_equal(p, expect)
    e, n = G.star(7)
    csr, _, level = run(e, n, 3)
    p = O.min_parents(csr, 3, level)
    assert p[3] == 3 and p[0] == 3 and all(p[v] == 0 for v in range(1, n) if v != 3)


def test_min_parents_is_a_valid_tree():
    scale = 11
    n = 1 << scale
    e = K.edges_host(scale)
    csr = O.build_csr(e, n)
    label = O.components(e, n)
    for r in K.select_roots(K.nonisolated_host(e, n), 4, K.root_seed(scale)):
        _, level = O.bfs(csr, r)
        p = O.min_parents(csr, r, level)
        assert O.validate(csr, r, p, level, label) == 0
        # no neighbour one level up has a smaller id than the chosen parent
        for v in np.flatnonzero(level > 0)[:300]:
            row = csr.row(v)
            cand = row[level[row] == level[v] - 1]
            assert p[v] == cand.min()
