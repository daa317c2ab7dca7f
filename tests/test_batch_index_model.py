"""The batched traversal's index arithmetic replayed on the CPU with every
array access bounds-checked (tests/batch_index_model.cpp models k_ms_seed,
the fills, td_phase, bu_phase with their hub pieces, hub_of, commit_atomic and
step_parents, and Kernel 1's hub list), on the 300,000-leaf star of the
batched hub-row test with that test's roots and on a Kronecker graph, in every
direction mode.  Its levels must equal the oracle's and its parents be valid,
so the model follows what the kernels compute."""
import os
import subprocess

import numpy as np
import pytest

import kronecker as K
import oracle as O
from tests import graphs as G

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def model(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("model") / "batch_index_model")
    subprocess.run(["g++", "-O2", "-std=c++17", "-o", exe,
                    os.path.join(HERE, "batch_index_model.cpp")], check=True)
    return exe


def run_model(exe, tmp, csr, roots, direction, alpha, parents, waves):
    rp = np.asarray(csr.row_ptr, dtype=np.int64)
    ci = np.asarray(csr.col_idx, dtype=np.int32)
    n = len(rp) - 1
    inp, out = str(tmp / "in.bin"), str(tmp / "out.bin")
    with open(inp, "wb") as f:
        f.write(np.array([n, len(ci)], dtype=np.int64).tobytes())
        f.write(rp.tobytes())
        f.write(ci.tobytes())
        f.write(np.array([len(roots)], dtype=np.int32).tobytes())
        f.write(np.array(roots, dtype=np.int64).tobytes())
    r = subprocess.run([exe, inp, str(direction), str(alpha), str(int(parents)), str(waves), out],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    raw = np.fromfile(out, dtype=np.uint8)
    k = len(roots)
    levels = raw[:k * n].view(np.int8).reshape(k, n)
    par = raw[k * n:].view(np.int32).reshape(k, n) if parents else None
    return levels, par


def check(exe, tmp, csr, roots, **kw):
    levels, par = run_model(exe, tmp, csr, roots, **kw)
    for b, r in enumerate(roots):
        _, want = O.bfs(csr, r)
        assert np.array_equal(levels[b].astype(np.int32), np.asarray(want)), (b, r, kw)
        if par is not None:
            assert O.check_parents(csr, r, par[b], np.asarray(want)) == 0, (b, r, kw)


MODES = [dict(direction=0, alpha=14.0), dict(direction=0, alpha=0.5), dict(direction=1, alpha=1.0),
         dict(direction=2, alpha=1.0)]


@pytest.mark.parametrize("mode", MODES, ids=["auto", "auto-early", "td", "bu"])
def test_star_300k(model, tmp_path, mode):
    leaves = 300_000
    e, n = G.star(leaves)
    extra = np.array([[1, 2], [3, 4]])
    csr = O.build_csr(np.concatenate([e, extra]), n)
    roots = [0, 1, 2, 5, leaves, leaves // 2]
    for parents in (True, False):
        check(model, tmp_path, csr, roots, parents=parents, waves=7, **mode)


@pytest.mark.parametrize("mode", MODES, ids=["auto", "auto-early", "td", "bu"])
def test_kronecker_scale12(model, tmp_path, mode):
    scale = 12
    e = K.edges_host(scale)
    csr = O.build_csr(e, 1 << scale)
    roots = K.select_roots(K.nonisolated_host(e, 1 << scale), 64, K.root_seed(scale))
    check(model, tmp_path, csr, roots, parents=True, waves=13, **mode)
