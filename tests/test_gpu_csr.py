"""Kernel 1 on the GPU: g5_build_csr bit-exact against the oracle CSR."""
import numpy as np
import pytest

import kronecker as K
from tests import golden
from tests.gpu_util import Case, to_dev

pytestmark = pytest.mark.gpu


def test_device_generator_matches_host():
    import torch
    for scale in (10, 16):
        d = K.edges_device(scale).cpu().numpy()
        assert np.array_equal(d, K.edges_host(scale))
        n = 1 << scale
        m = K.nonisolated_device(K.edges_device(scale), n).cpu().numpy()
        assert np.array_equal(m, K.nonisolated_host(K.edges_host(scale), n))
    torch.cuda.synchronize()


@pytest.mark.parametrize("scale", [8, 10, 14, 17, 20])
def test_kronecker_csr_bit_exact(scale):
    Case(K.edges_host(scale), 1 << scale).check_csr()


def test_golden_empty_rows():
    g = golden.load("csr_empty_rows.txt")
    c = Case(g["edges"], g["n"])
    c.check_csr()
    rp, ci = c.csr.arrays()
    assert rp.cpu().tolist() == g["row_ptr"].tolist()
    assert ci.cpu().tolist() == g["col_idx"].tolist()


def test_empty_edge_list():
    c = Case(np.zeros((0, 2), np.int64), 100)
    assert c.csr.nnz == 0
    c.check_csr()


def test_all_self_loops():
    e = np.stack([np.arange(50), np.arange(50)], 1)
    c = Case(e, 64)
    assert c.csr.nnz == 0
    c.check_csr()


def test_all_duplicates():
    e = np.tile(np.array([[3, 7]]), (5000, 1))
    e[::2] = [7, 3]
    c = Case(e, 9)
    assert c.csr.nnz == 2
    c.check_csr()


@pytest.mark.parametrize("n", [1, 2, 63, 65, 1000, 4097])
def test_odd_sizes(n):
    rng = np.random.default_rng(n)
    m = 3 * n
    e = rng.integers(0, n, size=(m, 2))
    Case(e, n).check_csr()


def test_trailing_and_leading_empty_rows():
    e = np.array([[10, 11], [11, 12], [12, 10]])
    Case(e, 40).check_csr()


def test_out_of_range_rejected():
    import paper_2012_13548_amd as g5
    for bad in ([[0, 5]], [[-1, 2]], [[2, 1 << 40]]):
        with pytest.raises(g5.G5Error) as ei:
            g5.build_csr(to_dev(np.array(bad)), 5)
        assert ei.value.status == g5.G5_EINVAL


def test_many_tiles_ragged():
    # 2m keys not a multiple of any tile size, several sort blocks
    rng = np.random.default_rng(5)
    n = 70001
    e = rng.integers(0, n, size=(1234567, 2))
    Case(e, n).check_csr()
