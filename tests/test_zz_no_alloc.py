"""g5_bfs_batch_noalloc (the batched traversal on the library's fixed
workspace) against g5_bfs_batch through the C-ABI: identical levels, valid
parents, on two calls in a row (the second on a smaller input), and the size
limit rejected cleanly."""
import numpy as np
import pytest

import kronecker as K
import oracle as O
import paper_2012_13548_amd as g5
from tests.gpu_util import Case

pytestmark = pytest.mark.gpu


def _check(case, roots):
    import torch
    pe, le = g5.bfs_batch(case.csr, roots)
    pn, ln = g5.bfs_batch_noalloc(case.csr, roots)
    assert torch.equal(ln, le)
    pn = pn.cpu().numpy()
    lv = ln.cpu().numpy()
    for b, r in enumerate(roots):
        _, olevel = O.bfs(case.ocsr, r)
        assert np.array_equal(lv[b].astype(np.int32), olevel), b
        assert O.validate(case.ocsr, r, pn[b], olevel, case.label) == 0, b
    _, lo = g5.bfs_batch_noalloc(case.csr, roots, parents=False)
    assert torch.equal(lo, le)


def test_noalloc_two_calls_then_smaller():
    scale = 20  # the largest graph the fixed workspace holds
    e = K.edges_host(scale)
    big = Case(e, 1 << scale)
    roots = K.select_roots(K.nonisolated_host(e, 1 << scale), 64, K.root_seed(scale))
    _check(big, roots)
    _check(big, roots[:17])
    scale = 12
    e = K.edges_host(scale)
    small = Case(e, 1 << scale)
    roots = K.select_roots(K.nonisolated_host(e, 1 << scale), 64, K.root_seed(scale))
    _check(small, roots[:40])


def test_noalloc_rejects_larger_graphs():
    import torch
    n = g5.NOALLOC_MAX_N + 1
    e = np.array([[0, 1], [1, n - 1]], dtype=np.int64)
    csr = g5.build_csr(torch.from_numpy(e).cuda(), n)
    with pytest.raises(g5.G5Error) as ei:
        g5.bfs_batch_noalloc(csr, [0])
    assert ei.value.status == g5.G5_EINVAL
