"""Full-size parity at the benchmark's configuration (Kronecker scale 26, edge
factor 16, the benchmark's roots and default launch parameters).

The oracle cannot afford everything at this size inside a test, so:
  * CSR: 2,000 sampled rows recomputed from the tuple list, bit-exact;
  * BFS: the tuple-list validator (levels are exactly hop distances and
    parents a BFS tree; proof in oracle.c) for 4 roots, and the oracle's own
    queue BFS, bit-exact on levels, for the first root;
  * batch: 64 roots at scale 22 (the batched configuration), every row equal
    to single-root levels, 8 rows bit-exact against the oracle.
"""
import numpy as np
import pytest

import kronecker as K
import oracle as O

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

SCALE = 26


@pytest.fixture(scope="module")
def big():
    import torch
    import paper_2012_13548_amd as g5
    n = 1 << SCALE
    dev_edges = K.edges_device(SCALE)
    csr = g5.build_csr(dev_edges, n)
    mask = K.nonisolated_device(dev_edges, n).cpu().numpy()
    roots = K.select_roots(mask, 64, K.root_seed(SCALE))
    # the device generator's tuples agree with the host generator's
    idx = np.random.default_rng(0).integers(0, dev_edges.shape[0], 100_000)
    sample_dev = dev_edges[torch.from_numpy(idx).cuda()].cpu().numpy()
    del dev_edges
    torch.cuda.empty_cache()
    host = K.edges_host(SCALE)
    assert np.array_equal(sample_dev, host[idx])
    return {"n": n, "csr": csr, "roots": roots, "edges": host}


def test_csr_sampled_rows(big):
    import torch
    n, csr, e = big["n"], big["csr"], big["edges"]
    rng = np.random.default_rng(1)
    rows = np.unique(rng.integers(0, n, 2000))
    lut = np.zeros(n, dtype=bool)
    lut[rows] = True
    u, w = e[:, 0], e[:, 1]
    loop = u == w
    hit0 = lut[u] & ~loop
    hit1 = lut[w] & ~loop
    src = np.concatenate([u[hit0], w[hit1]])
    dst = np.concatenate([w[hit0], u[hit1]])
    key = np.unique(src * n + dst)
    rp, ci = csr.arrays()
    rp_h = rp.cpu().numpy()
    assert rp_h[0] == 0 and rp_h[-1] == csr.nnz and np.all(np.diff(rp_h) >= 0)
    for v in rows:
        expect = key[(key >= v * n) & (key < (v + 1) * n)] - v * n
        got = ci[int(rp_h[v]):int(rp_h[v + 1])].cpu().numpy()
        assert np.array_equal(got, expect.astype(np.int32)), v
    del ci
    torch.cuda.empty_cache()


def test_bfs_validated_from_tuples(big):
    import paper_2012_13548_amd as g5
    for r in big["roots"][:4]:
        parent, level = g5.bfs(big["csr"], r)
        rule = O.validate_edges(big["edges"], big["n"], r, parent.cpu().numpy(),
                                level.cpu().numpy())
        assert rule == 0, f"root {r}: {O.RULES[rule]}"


def test_bfs_levels_equal_oracle(big):
    import paper_2012_13548_amd as g5
    r = big["roots"][0]
    _, level = g5.bfs(big["csr"], r)
    ocsr = O.build_csr(big["edges"], big["n"])
    _, olevel = O.bfs(ocsr, r)
    assert np.array_equal(level.cpu().numpy(), olevel)


def test_batch_scale22_64_roots():
    import torch
    import paper_2012_13548_amd as g5
    scale = 22
    n = 1 << scale
    e = K.edges_host(scale)
    csr = g5.build_csr(torch.from_numpy(e).cuda(), n)
    roots = K.select_roots(K.nonisolated_host(e, n), 64, K.root_seed(scale))
    parents, levels = g5.bfs_batch(csr, roots)
    for b, r in enumerate(roots):
        _, single = g5.bfs(csr, r)
        assert torch.equal(levels[b].to(torch.int32), single), b
    ocsr = O.build_csr(e, n)
    label = O.components(e, n)
    lv, pa = levels.cpu().numpy(), parents.cpu().numpy()
    for b in range(0, 64, 8):
        _, olevel = O.bfs(ocsr, roots[b])
        assert np.array_equal(lv[b].astype(np.int32), olevel)
        assert O.validate(ocsr, roots[b], pa[b], olevel, label) == 0
