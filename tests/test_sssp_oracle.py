"""Pins of the Kernel 3 oracle (Section 2.4, "Sequential SSSP"): the weighted
CSR, Dijkstra's distances and predecessors, the validator and the
deterministic predecessor choice, each against something other than itself:
closed forms on weighted paths, cycles, stars and grids; Floyd-Warshall by
brute force on small random multigraphs; scipy's Dijkstra on seeded
Kronecker graphs; and mutation tests for the validator."""
import numpy as np
import pytest

import kronecker as K
import oracle as O
from tests import graphs as G

INF = O.INF32


def run(e, w, n, src):
    csr = O.build_csr_w(e, w, n)
    dist, prev = O.sssp(csr, src)
    assert O.check_sssp(csr, src, dist, prev) == 0
    return csr, dist.astype(np.int64), prev


def min_weight_matrix(e, w, n):
    """Dense symmetric matrix of the smallest weight per vertex pair
    (np.inf where no tuple joins them), self-loops dropped."""
    a = np.full((n, n), np.inf)
    for (u, v), x in zip(e, w):
        if u != v:
            a[u, v] = min(a[u, v], x)
            a[v, u] = min(a[v, u], x)
    return a


def floyd_warshall(a):
    d = a.copy()
    np.fill_diagonal(d, 0)
    for k in range(d.shape[0]):
        d = np.minimum(d, d[:, k:k + 1] + d[k:k + 1, :])
    return d


def test_weighted_path_prefix_sums():
    rng = np.random.default_rng(1)
    n = 50
    e, _ = G.path(n)
    w = rng.integers(1, 256, n - 1).astype(np.uint8)
    pre = np.concatenate([[0], np.cumsum(w.astype(np.int64))])
    for r in (0, 17, n - 1):
        _, dist, prev = run(e, w, n, r)
        assert np.array_equal(dist, np.abs(pre - pre[r]))
        exp = np.arange(n) + np.where(np.arange(n) < r, 1, -1)
        exp[r] = r
        assert np.array_equal(prev, exp)


def test_weighted_cycle_both_ways():
    rng = np.random.default_rng(2)
    n = 31
    e, _ = G.cycle(n)
    w = rng.integers(1, 256, n).astype(np.uint8)  # edge i joins i and i+1 (mod n)
    cw = np.concatenate([[0], np.cumsum(w.astype(np.int64))])  # clockwise from 0
    total = cw[-1]
    _, dist, _ = run(e, w, n, 0)
    assert np.array_equal(dist, np.minimum(cw[:n], total - cw[:n]))


def test_star_and_leaf_root():
    rng = np.random.default_rng(3)
    leaves = 40
    e, n = G.star(leaves)
    w = rng.integers(1, 256, leaves).astype(np.uint8)  # edge to leaf i+1
    wl = np.concatenate([[0], w.astype(np.int64)])
    _, dist, prev = run(e, w, n, 0)
    assert np.array_equal(dist, wl)
    assert np.all(prev[1:] == 0)
    _, dist, prev = run(e, w, n, 5)
    exp = wl + wl[5]
    exp[0] = wl[5]
    exp[5] = 0
    assert np.array_equal(dist, exp)


@pytest.mark.parametrize("c", [1, 7, 255])
def test_uniform_grid_is_scaled_manhattan(c):
    a, b = 9, 13
    e, n = G.grid(a, b)
    w = np.full(len(e), c, np.uint8)
    for r in (0, 40, n - 1):
        csr, dist, _ = run(e, w, n, r)
        assert np.array_equal(dist, c * G.grid_dist(a, b, r))
    # deterministic predecessors from root 0: the neighbour above, else the one
    # to the left (the smaller id of the two tight neighbours)
    _, dist, _ = run(e, w, n, 0)
    mp = O.min_prev(csr, 0, dist.astype(np.uint32))
    v = np.arange(n)
    exp = np.where(v >= b, v - b, v - 1)
    exp[0] = 0
    assert np.array_equal(mp, exp)


def test_repeated_tuples_keep_the_smallest_weight():
    e = np.array([[0, 1], [1, 0], [0, 1], [1, 2], [2, 2]], np.int64)
    w = np.array([9, 5, 2, 4, 1], np.uint8)
    csr, dist, prev = run(e, w, 3, 0)
    assert csr.nnz == 4 and list(csr.row_weights(1)) == [2, 4]
    assert list(dist) == [0, 2, 6] and list(prev) == [0, 0, 1]


def test_unreached_and_zero_weights():
    e = np.array([[0, 1], [1, 2], [3, 4]], np.int64)
    w = np.array([0, 0, 3], np.uint8)
    _, dist, prev = run(e, w, 6, 1)
    assert list(dist) == [0, 0, 0, INF, INF, INF]
    assert list(prev) == [1, 1, 1, -1, -1, -1]


def test_floyd_warshall_random_multigraphs():
    rng = np.random.default_rng(4)
    for trial in range(300):
        n = int(rng.integers(1, 13))
        m = int(rng.integers(0, 3 * n + 1))
        e = rng.integers(0, n, (m, 2)).astype(np.int64)
        w = rng.integers(0 if trial % 3 == 0 else 1, 256, m).astype(np.uint8)
        fw = floyd_warshall(min_weight_matrix(e, w, n))
        for r in range(n):
            _, dist, prev = run(e, w, n, r)
            exp = np.where(np.isinf(fw[r]), INF, fw[r]).astype(np.int64)
            assert np.array_equal(dist, exp), (trial, r)


@pytest.mark.parametrize("scale", [10, 12])
def test_scipy_dijkstra_on_kronecker(scale):
    from scipy.sparse import coo_matrix
    from scipy.sparse.csgraph import dijkstra
    n = 1 << scale
    e = K.edges_host(scale)
    w = K.weights_host(scale)
    # symmetric, self-loops dropped, smallest weight per pair (numpy lexsort)
    keep = e[:, 0] != e[:, 1]
    u = np.concatenate([e[keep, 0], e[keep, 1]])
    v = np.concatenate([e[keep, 1], e[keep, 0]])
    x = np.concatenate([w[keep], w[keep]]).astype(np.int64)
    order = np.lexsort((x, v, u))
    u, v, x = u[order], v[order], x[order]
    first = np.ones(len(u), bool)
    first[1:] = (u[1:] != u[:-1]) | (v[1:] != v[:-1])
    mat = coo_matrix((x[first].astype(np.float64), (u[first], v[first])), shape=(n, n)).tocsr()
    csr = O.build_csr_w(e, w, n)
    assert np.array_equal(csr.row_ptr, mat.indptr)
    assert np.array_equal(csr.col_idx, mat.indices)
    assert np.array_equal(csr.weights, mat.data.astype(np.uint8))
    roots = K.select_roots(K.nonisolated_host(e, n), 8, K.root_seed(scale))
    ref = dijkstra(mat, directed=False, indices=roots)
    for i, r in enumerate(roots):
        dist, prev = O.sssp(csr, r)
        exp = np.where(np.isinf(ref[i]), INF, ref[i]).astype(np.int64)
        assert np.array_equal(dist.astype(np.int64), exp)
        assert O.check_sssp(csr, r, dist, prev) == 0
        assert O.check_sssp(csr, r, dist, O.min_prev(csr, r, dist)) == 0


@pytest.fixture(scope="module")
def kcase():
    scale = 11
    n = 1 << scale
    e = K.edges_host(scale)
    w = K.weights_host(scale)
    csr = O.build_csr_w(e, w, n)
    r = K.select_roots(K.nonisolated_host(e, n), 1, K.root_seed(scale))[0]
    dist, prev = O.sssp(csr, r)
    return csr, r, dist, prev


def test_validator_mutations(kcase):
    csr, r, dist, prev = kcase
    assert O.check_sssp(csr, r, dist, prev) == 0
    reached = np.flatnonzero((dist != INF) & (np.arange(csr.n) != r))
    v = int(reached[len(reached) // 2])
    d2 = dist.copy()
    d2[r] = 1
    assert O.check_sssp(csr, r, d2, prev) == 1
    p2 = prev.copy()
    p2[int(np.flatnonzero(dist == INF)[0])] = r
    assert O.check_sssp(csr, r, dist, p2) == 2
    nb = set(csr.row(v).tolist())
    p2 = prev.copy()
    p2[v] = next(u for u in reached if u not in nb)
    assert O.check_sssp(csr, r, dist, p2) == 3
    loose = [u for u, x in zip(csr.row(v), csr.row_weights(v))
             if dist[u] != INF and int(dist[u]) + int(x) != int(dist[v])]
    p2 = prev.copy()
    p2[v] = loose[0]
    assert O.check_sssp(csr, r, dist, p2) == 4
    # a distance one too large, with its predecessor still tight: some edge
    # into it shortens it (rule 5) or its children's rule 4 breaks
    d2 = dist.copy()
    leaf = next(x for x in reached if not np.any(prev == x))
    d2[leaf] += 1
    assert O.check_sssp(csr, r, d2, prev) in (4, 5)


def test_validator_rejects_prev_cycle():
    # zero-weight edges let two vertices point at each other with tight edges
    e = np.array([[0, 1], [1, 2], [2, 3], [3, 1]], np.int64)
    w = np.array([5, 0, 0, 0], np.uint8)
    csr = O.build_csr_w(e, w, 4)
    dist = np.array([0, 5, 5, 5], np.uint32)
    prev = np.array([0, 0, 3, 2], np.int32)
    assert O.check_sssp(csr, 0, dist, prev) == 6
    assert O.check_sssp(csr, 0, dist, np.array([0, 0, 1, 1], np.int32)) == 0
