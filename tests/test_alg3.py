"""The host experiment (the paper's parallel level-synchronous BFS with OpenMP
threads) against the oracle: levels bit-exact, parents valid by the oracle's
validator, for several thread counts; structured graphs with closed-form
levels; argument errors."""
import numpy as np
import pytest

import kronecker as K
import oracle as O
from paper_2012_13548_amd import alg3
from tests import graphs as G


def check(edges, n, roots, threads):
    csr = O.build_csr(edges, n)
    label = O.components(edges, n)
    for r in roots:
        parent, level, sec = alg3.bfs(csr.row_ptr, csr.col_idx, r, threads)
        _, olevel = O.bfs(csr, r)
        assert np.array_equal(level, olevel), (r, threads)
        assert O.validate(csr, r, parent, level, label) == 0, (r, threads)
        assert sec >= 0.0
    return csr


@pytest.mark.parametrize("threads", [1, 2, 4, 8])
@pytest.mark.parametrize("scale", [10, 13])
def test_kronecker(scale, threads):
    n = 1 << scale
    e = K.edges_host(scale)
    roots = K.select_roots(K.nonisolated_host(e, n), 4, K.root_seed(scale))
    check(e, n, [int(r) for r in roots], threads)


@pytest.mark.parametrize("threads", [1, 3, 8])
def test_structured(threads):
    e, n = G.path(300)
    csr = check(e, n, [0, 150], threads)
    _, level, _ = alg3.bfs(csr.row_ptr, csr.col_idx, 7, threads)
    assert np.array_equal(level, G.path_dist(300, 7))
    e, n = G.star(5000)
    check(e, n, [0, 17], threads)
    e, n = G.broom(300, 400)
    csr = check(e, n, [0], threads)
    _, level, _ = alg3.bfs(csr.row_ptr, csr.col_idx, 0, threads)
    assert np.array_equal(level, G.broom_dist(300, 400))
    # an isolated root reaches only itself
    e = np.array([[1, 2], [2, 3]], dtype=np.int64)
    csr = check(e, 6, [0, 5, 2], threads)


def test_errors():
    e, n = G.path(10)
    csr = O.build_csr(e, n)
    for root, threads in ((-1, 1), (n, 1), (0, 0)):
        with pytest.raises(ValueError):
            alg3.bfs(csr.row_ptr, csr.col_idx, root, threads)


def test_exports():
    # every function include/g5_alg3.h declares is exported by libg5alg3.so
    import ctypes
    import os
    import re
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    names = re.findall(r"\b(g5_alg3_\w+)\s*\(", open(os.path.join(root, "include", "g5_alg3.h")).read())
    assert names
    lib = ctypes.CDLL(alg3._LIB_PATH)
    for name in names:
        getattr(lib, name)
