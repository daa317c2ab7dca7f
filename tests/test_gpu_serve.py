"""Serving on the GPU: requests admitted while other batches run give the same
levels as the same request alone (bit-exact) and valid parents."""
import time

import numpy as np
import pytest

import kronecker as K
import oracle as O

pytestmark = pytest.mark.gpu


def test_mix_equals_alone():
    import torch
    import paper_2012_13548_amd as g5
    from paper_2012_13548_amd.serve import GpuExecutor, Server
    csrs, ocsr, labels, cands = {}, {}, {}, {}
    for s in (12, 14, 16):
        name = f"s{s}"
        e = K.edges_host(s)
        csrs[name] = g5.build_csr(torch.from_numpy(e).cuda(), 1 << s)
        ocsr[name] = O.build_csr(e, 1 << s)
        labels[name] = O.components(e, 1 << s)
        cands[name] = np.flatnonzero(K.nonisolated_host(e, 1 << s))
    ex = GpuExecutor(csrs, workers=3)
    srv = Server(ex, hbm_budget=8 << 30, workers=3).start()
    rng = np.random.default_rng(5)
    names = list(csrs)
    reqs = []
    for burst in range(12):
        for _ in range(int(rng.integers(1, 40))):
            g = names[int(rng.integers(0, 3))]
            reqs.append(srv.submit(g, int(rng.choice(cands[g]))))
        time.sleep(float(rng.uniform(0, 0.01)))
    assert srv.wait_all(len(reqs), timeout=300)
    srv.stop()
    assert srv.max_inflight >= 2, "batches never overlapped"
    assert any(r.batch_size and r.batch_size > 1 for r in reqs)
    for r in reqs:
        assert r.error is None, r.error
        level = r.level.to(torch.int32).cpu().numpy()
        _, alone = g5.bfs(csrs[r.graph], r.root)
        assert np.array_equal(level, alone.cpu().numpy()), (r.graph, r.root, r.batch_size)
        rule = O.validate(ocsr[r.graph], r.root, r.parent.cpu().numpy(), level, labels[r.graph])
        assert rule == 0, O.RULES[rule]
        _, olevel = O.bfs(ocsr[r.graph], r.root)
        assert np.array_equal(level, olevel)
        assert r.m_r == O.teps_edges(ocsr[r.graph], olevel)
    s = srv.summary()
    assert s["errors"] == 0 and s["p99_ms"] > 0
