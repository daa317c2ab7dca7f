"""Full-size parity at the benchmark's configuration (Kronecker scale 26, edge
factor 16, the benchmark's 64 roots and default launch parameters), and the
batched configuration (scale 22, 64 roots in one batch).

  * CSR: 2,000 sampled rows recomputed from the tuple list, bit-exact;
  * BFS: for every one of the 64 roots, the GPU's levels equal the oracle's
    queue BFS bit-exactly and its parent array passes the parent rules; the
    roots whose traversal takes a heavy top-down level are named from the
    direction log and must be among them; two roots (the first, and the first
    heavy one) also pass the tuple-list validator, which needs no CSR;
  * batch: all 64 rows bit-exact against the oracle, parents checked.

The oracle runs several roots at once from a thread pool (the C calls release
the interpreter lock).
"""
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import kronecker as K
import oracle as O

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

SCALE = 26
GROUP = 16  # roots per test: 64 roots in four tests


def _workers(cap=16):
    try:
        return max(1, min(cap, len(os.sched_getaffinity(0))))
    except AttributeError:
        return max(1, min(cap, os.cpu_count() or 1))


def _heavy_levels(info, nnz):
    """Levels the device ran as heavy top-down levels: top-down, frontier grew,
    more than nnz/2048 frontier edges (the library's default rule)."""
    out = []
    for i, d in enumerate(info["dir"]):
        grew = i > 0 and info["frontier"][i] > info["frontier"][i - 1]
        if d == 1 and grew and info["edges"][i] > nnz // 2048:
            out.append(i)
    return out


@pytest.fixture(scope="module")
def big():
    import torch
    import paper_2012_13548_amd as g5
    n = 1 << SCALE
    print(f"[fullsize] scale {SCALE}: device tuples, CSR", flush=True)
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
    print("[fullsize] oracle CSR", flush=True)
    ocsr = O.build_csr(host, n)
    heavy = {}
    for r in roots:
        _, _, info = g5.bfs(csr, r, stats=True)
        lv = _heavy_levels(info, csr.nnz)
        if lv:
            heavy[r] = lv
    print(f"[fullsize] {len(heavy)} of 64 roots run heavy top-down levels", flush=True)
    return {"n": n, "csr": csr, "roots": roots, "edges": host, "ocsr": ocsr, "heavy": heavy}


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
    assert np.array_equal(rp_h, big["ocsr"].row_ptr)
    for v in rows:
        expect = key[(key >= v * n) & (key < (v + 1) * n)] - v * n
        got = ci[int(rp_h[v]):int(rp_h[v + 1])].cpu().numpy()
        assert np.array_equal(got, expect.astype(np.int32)), v
    del ci
    torch.cuda.empty_cache()


def test_heavy_roots_present(big):
    # the heavy top-down path is exercised at full size (and all 64 roots,
    # these included, are compared with the oracle below)
    assert len(big["heavy"]) >= 1, "no root of the benchmark runs a heavy top-down level"


@pytest.mark.parametrize("group", range(64 // GROUP))
def test_bfs_levels_equal_oracle(big, group):
    import paper_2012_13548_amd as g5
    roots = big["roots"][group * GROUP:(group + 1) * GROUP]
    gpu = []
    for r in roots:
        parent, level = g5.bfs(big["csr"], r)
        gpu.append((parent.cpu().numpy(), level.cpu().numpy()))
        del parent, level
    print(f"[fullsize] group {group}: oracle BFS of {len(roots)} roots", flush=True)
    with ThreadPoolExecutor(_workers()) as ex:
        olevels = list(ex.map(lambda r: O.bfs(big["ocsr"], r)[1], roots))
    for r, (parent, level), olevel in zip(roots, gpu, olevels):
        bad = np.flatnonzero(level != olevel)
        tag = f"root {r}{' (heavy levels %s)' % big['heavy'][r] if r in big['heavy'] else ''}"
        assert bad.size == 0, (f"{tag}: {bad.size} levels differ, first at {bad[:5]}: "
                               f"gpu {level[bad[:5]]} oracle {olevel[bad[:5]]}")
        rule = O.check_parents(big["ocsr"], r, parent, level)
        assert rule == 0, f"{tag}: parent array invalid ({O.RULES[rule]})"


def test_bfs_validated_from_tuples(big):
    import paper_2012_13548_amd as g5
    picks = [big["roots"][0]]
    if big["heavy"]:
        picks.append(next(iter(big["heavy"])))
    for r in picks:
        parent, level = g5.bfs(big["csr"], r)
        rule = O.validate_edges(big["edges"], big["n"], r, parent.cpu().numpy(),
                                level.cpu().numpy())
        assert rule == 0, f"root {r}: {O.RULES[rule]}"


def test_batch_scale22_64_roots():
    import torch
    import paper_2012_13548_amd as g5
    scale = 22
    n = 1 << scale
    e = K.edges_host(scale)
    csr = g5.build_csr(torch.from_numpy(e).cuda(), n)
    roots = K.select_roots(K.nonisolated_host(e, n), 64, K.root_seed(scale))
    parents, levels = g5.bfs_batch(csr, roots)
    lv, pa = levels.cpu().numpy(), parents.cpu().numpy()
    ocsr = O.build_csr(e, n)
    with ThreadPoolExecutor(_workers()) as ex:
        olevels = list(ex.map(lambda r: O.bfs(ocsr, r)[1], roots))
    for b, (r, olevel) in enumerate(zip(roots, olevels)):
        bad = np.flatnonzero(lv[b].astype(np.int32) != olevel)
        assert bad.size == 0, f"row {b} root {r}: {bad.size} levels differ, first {bad[:5]}"
        rule = O.check_parents(ocsr, r, pa[b], olevel)
        assert rule == 0, f"row {b} root {r}: parents invalid ({O.RULES[rule]})"
