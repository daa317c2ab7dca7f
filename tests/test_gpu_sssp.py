"""Kernel 3 on the GPU (delta-stepping through the C-ABI) against the oracle
(Dijkstra, Section 2.4): the weighted CSR bit-exact (smallest weight of
repeated tuples), distances bit-exact, predecessors equal to the oracle's
deterministic choice and valid by the independent validator."""
import numpy as np
import pytest

import kronecker as K
import oracle as O
import paper_2012_13548_amd as g5
from tests import graphs as G

pytestmark = pytest.mark.gpu


class WCase:
    def __init__(self, edges, weights, n):
        import torch
        self.edges = np.ascontiguousarray(edges, dtype=np.int64).reshape(-1, 2)
        self.weights = np.ascontiguousarray(weights, dtype=np.uint8)
        self.n = n
        self.csr = g5.build_csr_w(torch.from_numpy(self.edges).cuda(),
                                  torch.from_numpy(self.weights).cuda(), n)
        self.ocsr = O.build_csr_w(self.edges, self.weights, n)

    def check_csr(self):
        rp, ci = self.csr.arrays()
        assert np.array_equal(rp.cpu().numpy(), self.ocsr.row_ptr)
        assert np.array_equal(ci.cpu().numpy(), self.ocsr.col_idx)
        assert np.array_equal(self.csr.weights().cpu().numpy(), self.ocsr.weights)

    def check(self, src, **kw):
        dist, prev, info = g5.sssp(self.csr, src, stats=True, **kw)
        dist = dist.cpu().numpy().view(np.uint32)
        prev = prev.cpu().numpy()
        odist, _ = O.sssp(self.ocsr, src)
        bad = np.flatnonzero(dist != odist)
        assert bad.size == 0, (f"source {src} {kw}: {bad.size} distances differ, first "
                               f"{bad[:5]}: gpu {dist[bad[:5]]} oracle {odist[bad[:5]]}")
        assert np.array_equal(prev, O.min_prev(self.ocsr, src, odist)), (src, kw)
        rule = O.check_sssp(self.ocsr, src, dist, prev)
        assert rule == 0, f"source {src} {kw}: {O.SSSP_RULES[rule]}"
        return dist, prev, info


@pytest.fixture(scope="module", params=[10, 16])
def kron(request):
    scale = request.param
    n = 1 << scale
    e = K.edges_host(scale)
    c = WCase(e, K.weights_host(scale), n)
    roots = K.select_roots(K.nonisolated_host(e, n), 8, K.root_seed(scale))
    return c, roots


def test_weighted_csr_bit_exact(kron):
    kron[0].check_csr()


@pytest.mark.parametrize("delta", [None, 1, 8, 255, 1 << 20])
def test_kronecker_distances(kron, delta):
    c, roots = kron
    for r in roots[:4] if delta else roots:
        c.check(r, delta=delta)


@pytest.mark.parametrize("pull_div", [-1, 2, 1_000_000])
def test_kronecker_pull(kron, pull_div):
    # never pull; pull the rounds holding half the edges; pull every round
    c, roots = kron
    pulls = 0
    for r in roots:
        _, _, info = c.check(r, pull_div=pull_div)
        pulls += info["pulls"]
    assert (pulls == 0) if pull_div < 0 else (pull_div < 1000 or pulls > 0)


def test_kronecker_scale20():
    scale = 20
    n = 1 << scale
    e = K.edges_host(scale)
    c = WCase(e, K.weights_host(scale), n)
    c.check_csr()
    roots = K.select_roots(K.nonisolated_host(e, n), 4, K.root_seed(scale))
    for r in roots:
        _, _, info = c.check(r)
        assert info["rounds"] > 0 and info["buckets"] >= 1


def test_structured():
    rng = np.random.default_rng(7)
    cases = []
    e, n = G.path(3000)  # many buckets and rounds
    cases.append((e, rng.integers(1, 256, len(e)), n, [0, 1500]))
    e, n = G.grid(40, 70)
    cases.append((e, np.full(len(e), 3), n, [0, 1234]))
    e, n = G.star(300_000)  # the centre's row is relaxed in hub pieces
    cases.append((e, rng.integers(1, 256, len(e)), n, [0, 7, n - 1]))
    parts = G.disjoint_union(G.path(40), G.star(70), G.cycle(11))
    e, n = parts[0], parts[1]
    cases.append((e, rng.integers(0, 3, len(e)), n + 2, [0, 45, n + 1]))  # zero weights, isolated
    for e, w, n, roots in cases:
        c = WCase(e, w.astype(np.uint8), n)
        c.check_csr()
        for r in roots:
            for delta in (None, 4):
                c.check(r, delta=delta)
            # every round pulled: hub rows in pieces, rows by lane and by wavefront
            c.check(r, pull_div=1_000_000)


def test_repeated_tuples_and_loops():
    e = np.array([[0, 1], [1, 0], [0, 1], [1, 2], [2, 2], [2, 3], [3, 2]], np.int64)
    w = np.array([9, 5, 2, 4, 1, 200, 7], np.uint8)
    c = WCase(e, w, 5)
    c.check_csr()
    dist, prev, _ = c.check(0)
    assert list(dist[:4]) == [0, 2, 6, 13] and dist[4] == O.INF32


def test_errors():
    import torch
    e = torch.tensor([[0, 1]], dtype=torch.int64).cuda()
    plain = g5.build_csr(e, 4)
    with pytest.raises(g5.G5Error) as ei:
        g5.sssp(plain, 0)
    assert ei.value.status == g5.G5_EINVAL
    c = WCase(np.array([[0, 1]]), np.array([3]), 4)
    for bad in (-1, 4):
        with pytest.raises(g5.G5Error) as ei:
            g5.sssp(c.csr, bad)
        assert ei.value.status == g5.G5_EINVAL
    # the BFS path runs on a weighted graph too
    _, lv = g5.bfs(c.csr, 0)
    assert lv.cpu().tolist() == [0, 1, -1, -1]
