"""Kernel 2 on the GPU: g5_bfs levels bit-exact against the oracle, parents
valid by the oracle's validator, for every direction policy and claim mode."""
import numpy as np
import pytest

import kronecker as K
import paper_2012_13548_amd as g5
from tests import golden
from tests import graphs as G
from tests.gpu_util import Case

pytestmark = pytest.mark.gpu

MODES = [dict(direction=g5.DIR_AUTO), dict(direction=g5.DIR_TOPDOWN),
         dict(direction=g5.DIR_BOTTOMUP), dict(direction=g5.DIR_AUTO, claim=g5.CLAIM_CAS),
         dict(direction=g5.DIR_AUTO, alpha=1e6, beta=1e6),
         dict(direction=g5.DIR_AUTO, alpha=1e-3, beta=2.0), dict(hint=False),
         dict(direction=g5.DIR_BOTTOMUP, hint=False, lane_scan=1),
         dict(packed=True), dict(direction=g5.DIR_BOTTOMUP, packed=True, hint=False, lane_scan=1),
         dict(lds=False), dict(direction=g5.DIR_BOTTOMUP, lds=False, packed=True),
         dict(direction=g5.DIR_BOTTOMUP, lds_kb=16, lds_density=1.0, packed=True),
         dict(direction=g5.DIR_BOTTOMUP, lds_kb=16, lds_density=1.0, packed=False),
         dict(vertices_per_lane=2), dict(direction=g5.DIR_BOTTOMUP, vertices_per_lane=2, packed=True),
         dict(direction=g5.DIR_BOTTOMUP, vertices_per_lane=2, lds_density=1.0, lane_scan=16),
         dict(gamma=0.5, alpha=2.0)]
MODE_IDS = ["auto", "td", "bu", "auto-cas", "auto-eager", "auto-late", "nohint", "bu-nohint-1",
            "packed", "bu-packed-nohint-1", "nolds", "bu-nolds-packed", "bu-lds16-packed",
            "bu-lds16-rows", "vpl2", "bu-vpl2-packed", "bu-vpl2-lds-16", "gamma-early"]


@pytest.fixture(params=range(len(MODES)), ids=MODE_IDS)
def mode(request):
    return MODES[request.param]


def structured():
    out = {}
    out["path"] = G.path(300)
    out["star"] = G.star(5000)
    out["grid"] = G.grid(37, 41)
    out["cycle"] = G.cycle(257)
    out["complete"] = G.complete(40)
    out["tree"] = G.binary_tree(10)
    e, n, _ = G.disjoint_union(G.path(70), G.cycle(9), G.star(130))
    out["union"] = (e, n + 5)
    return out


@pytest.fixture(scope="module")
def cases():
    return {k: Case(*v) for k, v in structured().items()}


@pytest.mark.parametrize("name", list(structured().keys()))
def test_structured(cases, name, mode):
    c = cases[name]
    rng = np.random.default_rng(len(name))
    for r in [0, c.n - 1] + list(rng.integers(0, c.n, 3)):
        c.check_root(int(r), **mode)


@pytest.mark.parametrize("name", ["fail1.txt", "two_components.txt"])
def test_golden(name, mode):
    g = golden.load(name)
    c = Case(g["edges"], g["n"])
    parent, level = c.check_root(g["root"], **mode)
    for v, l in g["level"].items():
        assert level[v] == l
    for v, ch in g["parent_choices"].items():
        assert parent[v] in ch


def test_isolated_root(mode):
    c = Case(np.array([[1, 2], [2, 3]]), 70)
    parent, level = c.check_root(0, **mode)
    assert (level >= 0).sum() == 1 and parent[0] == 0
    c.check_root(69, **mode)


@pytest.mark.parametrize("leaves", [100_000, 1_000_000])
def test_hub_star(leaves):
    # one row split over ~1000 top-down blocks
    e, n = G.star(leaves)
    c = Case(e, n)
    for m in (dict(direction=g5.DIR_TOPDOWN), dict(direction=g5.DIR_AUTO),
              dict(direction=g5.DIR_BOTTOMUP)):
        c.check_root(0, **m)
        c.check_root(leaves // 2, **m)


def test_long_path():
    # 10,000 levels; relabelled so consecutive levels are far apart in memory
    e, n, perm = G.long_path_relabelled(10_000, 3)
    c = Case(e, n)
    for m in (dict(direction=g5.DIR_AUTO), dict(direction=g5.DIR_TOPDOWN)):
        c.check_root(int(perm[0]), **m)
        c.check_root(int(perm[n // 2]), **m)


def test_deep_switch_to_bottom_up():
    # The frontier first grows at level 300 (a path, then a star whose 4,000
    # leaves each hold a pendant vertex), so the switch to bottom-up comes after
    # the byte levels were widened: its frontier bitmap is built from the int32
    # levels, and min-id claims test the int32 level of a target.
    e, n = G.broom(300, 4000)
    c = Case(e, n)
    want = G.broom_dist(300, 4000)
    for m in (dict(), dict(claim=g5.CLAIM_CAS), dict(min_parent=True), dict(hint=False),
              dict(lds=False), dict(direction=g5.DIR_TOPDOWN, min_parent=True)):
        parent, level = c.check_root(0, **m)
        assert np.array_equal(level, want), m
        assert np.array_equal(parent[300 + 4000:], np.arange(300, 300 + 4000)), m


def comb(seed=3):
    """Rows the packed bottom-up scan resolves a few entries in, beside long rows
    it never resolves: vertex 100 is the root; even-numbered vertices from 1101
    on hold 3 smaller-id leaves, the root, then 150 larger-id leaves; odd ones
    hold 253 leaves and not the root, so a wavefront's layout interleaves both
    and the scan must jump past the resolved rows' remaining entries."""
    rng = np.random.default_rng(seed)
    lo, root, hi, first = np.arange(0, 100), 100, np.arange(101, 1101), 1101
    edges = []
    for k in range(400):
        v = first + k
        nb = [rng.choice(lo, 3, replace=False)]
        nb += [[root], rng.choice(hi, 150, replace=False)] if k % 2 == 0 else \
              [rng.choice(hi, 250, replace=False)]
        edges += [(v, int(u)) for u in np.concatenate(nb)]
    return np.array(edges, dtype=np.int64), first + 400, root


@pytest.mark.parametrize("m", [dict(direction=g5.DIR_BOTTOMUP, packed=True, hint=False, lane_scan=1),
                               dict(direction=g5.DIR_BOTTOMUP, packed=True, hint=False, lane_scan=4),
                               dict(direction=g5.DIR_BOTTOMUP, packed=True, lane_scan=2, lds=False),
                               dict(direction=g5.DIR_BOTTOMUP, packed=True, lds_density=1.0),
                               dict(direction=g5.DIR_BOTTOMUP, packed=True, vertices_per_lane=2),
                               dict(direction=g5.DIR_AUTO, packed=True)],
                         ids=["bu-1", "bu-4", "bu-nolds-2", "bu-lds", "bu-vpl2", "auto"])
def test_packed_scan_resolved_rows(m):
    import oracle as O
    e, n, root = comb()
    c = Case(e, n)
    for r in (root, n - 1, 0):
        c.check_root(r, **m)
        parent, level = c.check_root(r, min_parent=True, **m)
        assert np.array_equal(parent, O.min_parents(c.ocsr, r, level)), (r, m)


@pytest.fixture(scope="module")
def kron10():
    scale = 10
    e = K.edges_host(scale)
    c = Case(e, 1 << scale)
    roots = K.select_roots(K.nonisolated_host(e, 1 << scale), 8, K.root_seed(scale))
    return c, roots


def test_kronecker_scale10_all_roots(kron10, mode):
    c, roots = kron10
    for r in roots:
        c.check_root(r, **mode)


@pytest.mark.parametrize("lane_scan", [1, 2, 4, 8, 16])
def test_lane_scan_variants(kron10, lane_scan):
    c, roots = kron10
    for r in roots[:3]:
        c.check_root(r, lane_scan=lane_scan)


@pytest.mark.parametrize("td_blocks_per_cu", [1, 3, 17])
@pytest.mark.parametrize("direction", [g5.DIR_TOPDOWN, g5.DIR_AUTO])
def test_expansion_grid_variants(kron16, td_blocks_per_cu, direction):
    # tiles advance over the frontier's edges in grid-stride rounds; a small grid
    # takes many rounds per workgroup, so every tile's appends share the queue's
    # packed counter across rounds
    c, roots = kron16
    for r in roots[:3]:
        c.check_root(r, direction=direction, td_blocks_per_cu=td_blocks_per_cu)


@pytest.mark.parametrize("heavy_kedges", [-1, 1, 0])
def test_heavy_levels(kron16, heavy_kedges):
    # heavy top-down levels claim without reading the claimed vertices' row
    # offsets and send the next level bottom-up: off, on almost every growing
    # level (1,000 edges), and the default threshold
    c, roots = kron16
    for r in roots:
        c.check_root(r, heavy_kedges=heavy_kedges)
        c.check_root(r, heavy_kedges=heavy_kedges, claim=g5.CLAIM_CAS)
        c.check_root(r, heavy_kedges=heavy_kedges, min_parent=True)


def test_heavy_hub_star():
    # a star of 200,000 leaves (plus a few leaf-leaf edges) from a leaf with a
    # leaf neighbour: level 1 is the hub and that neighbour (a growing
    # frontier), level 2 claims every other leaf in one heavy top-down level
    # (alpha and gamma keep it top-down); from a plain leaf it is not heavy
    e, n = G.star(200_000)
    extra = np.array([[1, 2], [3, 4], [5, 6]])
    c = Case(np.concatenate([e, extra]), n)
    for r in (1, 4, 5, 7, n - 1):
        _, _, st = g5.bfs(c.csr, r, stats=True, heavy_kedges=1, alpha=1e-3, gamma=-1)
        # from a leaf with a leaf neighbour level 1 is heavy; from a plain leaf the
        # hub alone is level 1 (not a growing frontier) and level 2 goes bottom-up
        assert st["heavy_mask"] == (0b10 if r <= 6 else 0), (r, st["dir"], st["heavy_mask"])
        c.check_root(r, heavy_kedges=1, alpha=1e-3, gamma=-1)


@pytest.fixture(scope="module")
def kron16():
    scale = 16
    e = K.edges_host(scale)
    c = Case(e, 1 << scale)
    roots = K.select_roots(K.nonisolated_host(e, 1 << scale), 8, K.root_seed(scale))
    return c, roots


def test_kronecker_scale16(kron16, mode):
    c, roots = kron16
    for r in roots:
        c.check_root(r, **mode)


def test_kronecker_scale20_64_roots():
    scale = 20
    n = 1 << scale
    e = K.edges_host(scale)
    c = Case(e, n)
    roots = K.select_roots(K.nonisolated_host(e, n), 64, K.root_seed(scale))
    dirs = set()
    for r in roots:
        c.check_root(r)
        _, _, st = g5.bfs(c.csr, r, stats=True)
        dirs |= set(st["dir"])
    assert dirs == {1, 2}, "direction-optimising run never switched"
    for r in roots[:4]:
        c.check_root(r, direction=g5.DIR_TOPDOWN)
        c.check_root(r, direction=g5.DIR_BOTTOMUP)


def test_repeat_stable(kron10):
    c, roots = kron10
    first = None
    for _ in range(10):
        _, level = g5.bfs(c.csr, roots[0])
        level = level.cpu().numpy()
        if first is None:
            first = level
        assert np.array_equal(level, first)


def test_bad_root(kron10):
    c, _ = kron10
    for r in (-1, c.n, 1 << 40):
        with pytest.raises(g5.G5Error) as ei:
            g5.bfs(c.csr, r)
        assert ei.value.status == g5.G5_EINVAL


def test_unaligned_outputs(kron10):
    import torch
    c, roots = kron10
    buf = torch.empty(2 * c.n + 2, dtype=torch.int32, device="cuda:0")
    parent, level = g5.bfs(c.csr, roots[1], parent=buf[1:c.n + 1], level=buf[c.n + 1:2 * c.n + 1])
    _, ref = g5.bfs(c.csr, roots[1])
    assert torch.equal(level, ref)


@pytest.mark.parametrize("direction", [g5.DIR_AUTO, g5.DIR_TOPDOWN, g5.DIR_BOTTOMUP])
@pytest.mark.parametrize("packed", [False, True])
def test_min_parent_bit_exact(kron16, direction, packed):
    import oracle as O
    c, roots = kron16
    for r in roots[:4]:
        parent, level = c.check_root(r, direction=direction, packed=packed, min_parent=True)
        assert np.array_equal(parent, O.min_parents(c.ocsr, r, level))


def test_min_parent_structured(cases):
    import oracle as O
    for name in ("grid", "tree", "union", "star"):
        c = cases[name]
        for r in (0, c.n // 3):
            for d in (g5.DIR_AUTO, g5.DIR_TOPDOWN, g5.DIR_BOTTOMUP):
                parent, level = c.check_root(r, direction=d, min_parent=True)
                assert np.array_equal(parent, O.min_parents(c.ocsr, r, level)), (name, r, d)
