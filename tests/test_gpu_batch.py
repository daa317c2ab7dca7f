"""Batched multi-source BFS on the GPU: every row of g5_bfs_batch bit-exact
against the oracle's single-root levels (as int8), parents valid."""
import numpy as np
import pytest

import kronecker as K
import oracle as O
import paper_2012_13548_amd as g5
from tests import graphs as G
from tests.gpu_util import Case, check_batch

pytestmark = pytest.mark.gpu

MODES = [dict(), dict(direction=g5.DIR_TOPDOWN), dict(direction=g5.DIR_BOTTOMUP),
         dict(alpha=1e-3), dict(alpha=1e6), dict(parents=False), dict(persistent=True),
         dict(persistent=True, parents=False, direction=g5.DIR_BOTTOMUP), dict(graph=True),
         dict(graph=True, parents=False, direction=g5.DIR_TOPDOWN)]
MODE_IDS = ["auto", "td", "bu", "auto-bu-early", "auto-td-long", "levels-only", "persistent",
            "persistent-bu-levels", "graph", "graph-td-levels"]


@pytest.fixture(params=range(len(MODES)), ids=MODE_IDS)
def mode(request):
    return dict(MODES[request.param])


@pytest.fixture(scope="module")
def kron12():
    scale = 12
    e = K.edges_host(scale)
    c = Case(e, 1 << scale)
    roots = K.select_roots(K.nonisolated_host(e, 1 << scale), 64, K.root_seed(scale))
    return c, roots


@pytest.mark.parametrize("k", [1, 7, 63, 64])
def test_kronecker_scale12(kron12, k, mode):
    c, roots = kron12
    check_batch(c, roots[:k], **mode)


def test_duplicate_roots(kron12, mode):
    c, roots = kron12
    check_batch(c, [roots[0], roots[1], roots[0], roots[0], roots[2], roots[1]], **mode)


@pytest.mark.parametrize("name", ["grid", "cycle", "tree", "union"])
def test_structured(name, mode):
    builders = {"grid": lambda: G.grid(23, 29), "cycle": lambda: G.cycle(201),
                "tree": lambda: G.binary_tree(9),
                "union": lambda: G.disjoint_union(G.path(40), G.star(70), G.cycle(11))[:2]}
    e, n = builders[name]()
    c = Case(e, n + 3)
    rng = np.random.default_rng(11)
    roots = [int(x) for x in rng.integers(0, n + 3, 40)]
    check_batch(c, roots, **mode)


@pytest.mark.parametrize("leaves", [20_000, 300_000])
def test_hub_rows(leaves, mode):
    # the centre's row is split into kHubChunk pieces; roots at leaves and centre
    e, n = G.star(leaves)
    extra = np.array([[1, 2], [3, 4]])  # a few leaf-leaf edges
    c = Case(np.concatenate([e, extra]), n)
    roots = [0, 1, 2, 5, leaves, leaves // 2]
    check_batch(c, roots, **mode)


def test_isolated_roots():
    c = Case(np.array([[1, 2], [2, 3]]), 200)
    check_batch(c, [0, 5, 1, 199])


def test_depth_limit():
    # int8 levels hold up to 127: a path of 255 vertices from its middle fits
    # exactly; on 256 vertices every root has eccentricity >= 128 and the call
    # reports G5_ERANGE
    e, n = G.path(255)
    c = Case(e, n)
    _, lv, _ = check_batch(c, [127])
    assert lv.max() == 127
    # the graph path: 128 levels are 16 replays of its 8-level graph
    _, lv, info = check_batch(c, [127, 127], graph=True)
    assert lv.max() == 127 and info["nlevels"] == 128
    for roots in ([126], [0, 127]):
        for mode in (dict(), dict(persistent=True), dict(graph=True)):
            with pytest.raises(g5.G5Error) as ei:
                g5.bfs_batch(c.csr, roots, **mode)
            assert ei.value.status == g5.G5_ERANGE
    e, n = G.path(256)
    c = Case(e, n)
    for roots in ([127], [128], [0, 127]):
        with pytest.raises(g5.G5Error) as ei:
            g5.bfs_batch(c.csr, roots)
        assert ei.value.status == g5.G5_ERANGE


def test_bad_arguments(kron12):
    c, roots = kron12
    for bad in ([], list(range(65)), [-1], [c.n]):
        with pytest.raises(g5.G5Error) as ei:
            g5.bfs_batch(c.csr, bad)
        assert ei.value.status == g5.G5_EINVAL


@pytest.mark.parametrize("scale", [16, 20])
def test_kronecker_64_roots(scale):
    n = 1 << scale
    e = K.edges_host(scale)
    c = Case(e, n)
    roots = K.select_roots(K.nonisolated_host(e, n), 64, K.root_seed(scale))
    _, _, info = check_batch(c, roots)
    assert set(info["dir"]) == {1, 2}, info
    # same levels as 64 single-root calls
    import torch
    _, lv = g5.bfs_batch(c.csr, roots[:8], parents=False)
    for b, r in enumerate(roots[:8]):
        _, l1 = g5.bfs(c.csr, r)
        assert torch.equal(lv[b].to(torch.int32), l1)


def test_repeat_stable(kron12):
    c, roots = kron12
    ref = None
    for _ in range(5):
        _, lv = g5.bfs_batch(c.csr, roots, parents=False)
        lv = lv.cpu().numpy()
        if ref is None:
            ref = lv
        assert np.array_equal(lv, ref)


def test_graph_replays_between_eager_work(kron12):
    # one instantiated graph serves batches with different roots, k and output
    # buffers; eager launches and synchronisations run between the replays,
    # and every result equals the stepped (eager) launch's
    import torch
    c, roots = kron12
    for i, k in enumerate([64, 5, 64, 1, 33]):
        rs = roots[i:i + k] if i + k <= len(roots) else roots[:k]
        pe, le = g5.bfs_batch(c.csr, rs)
        torch.cuda.synchronize()
        pg, lg = g5.bfs_batch(c.csr, rs, graph=True)
        assert torch.equal(lg, le), (i, k)
        _, lo = g5.bfs_batch(c.csr, rs, parents=False, graph=True)
        assert torch.equal(lo, le), (i, k)
        pg, lg = pg.cpu().numpy(), lg.cpu().numpy()
        for b, r in enumerate(rs):
            rule = O.validate(c.ocsr, r, pg[b], lg[b].astype(np.int32), c.label)
            assert rule == 0, (i, k, b)
