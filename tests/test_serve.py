"""Serving scheduler on the CPU: an oracle-backed executor stands in for the GPU
so admission, coalescing, concurrency and fallback logic run without a device."""
import threading
import time

import numpy as np
import pytest

import kronecker as K
import oracle as O
from paper_2012_13548_amd.serve import RangeExceeded, Server
from tests import graphs as G


class OracleExecutor:
    def __init__(self, graphs, delay=0.0, range_limit=None):
        self.ocsr = {k: O.build_csr(e, n) for k, (e, n) in graphs.items()}
        self.graphs = {k: n for k, (e, n) in graphs.items()}
        self.delay = delay
        self.range_limit = range_limit
        self.lock = threading.Lock()
        self.active = self.max_active = 0
        self.calls = []

    def footprint(self, g, k):
        n = self.graphs[g]
        return k * n * 5 + 32 * n

    def run(self, g, roots, wid, single=False):
        with self.lock:
            self.active += 1
            self.max_active = max(self.max_active, self.active)
            self.calls.append((g, len(roots), wid, single))
        try:
            time.sleep(self.delay)
            c = self.ocsr[g]
            levels = np.empty((len(roots), c.n), np.int32)
            parents = np.empty((len(roots), c.n), np.int32)
            for i, r in enumerate(roots):
                parents[i], levels[i] = O.bfs(c, r)
            if (self.range_limit is not None and len(roots) > 1
                    and levels.max() > self.range_limit):
                raise RangeExceeded("level too deep for a batch")
            return parents, levels
        finally:
            with self.lock:
                self.active -= 1

    def edges(self, g, level_rows, wid):
        return [O.teps_edges(self.ocsr[g], lv) for lv in level_rows]


@pytest.fixture(scope="module")
def pool():
    out = {}
    for s in (8, 10):
        out[f"s{s}"] = (K.edges_host(s), 1 << s)
    out["path"] = G.path(300)
    return out


def roots_for(pool, g, k, seed=0):
    e, n = pool[g]
    mask = K.nonisolated_host(e, n)
    rng = np.random.default_rng(seed)
    return [int(x) for x in rng.choice(np.flatnonzero(mask), size=k)]


def check_results(ex, reqs):
    for r in reqs:
        assert r.error is None, r.error
        _, lv = O.bfs(ex.ocsr[r.graph], r.root)
        assert np.array_equal(r.level, lv)
        e = ex.ocsr[r.graph]
        assert r.m_r == O.teps_edges(e, lv)


def test_all_complete_and_correct(pool):
    ex = OracleExecutor(pool)
    srv = Server(ex, hbm_budget=1 << 40, workers=2).start()
    reqs = [srv.submit(g, r) for g in ("s8", "s10") for r in roots_for(pool, g, 20)]
    assert srv.wait_all(len(reqs), timeout=60)
    srv.stop()
    check_results(ex, reqs)
    s = srv.summary()
    assert s["requests"] == 40 and s["errors"] == 0 and s["p99_ms"] >= s["p50_ms"] >= 0


def test_coalescing_up_to_64(pool):
    ex = OracleExecutor(pool)
    srv = Server(ex, hbm_budget=1 << 40, workers=1)
    reqs = [srv.submit("s10", r) for r in roots_for(pool, "s10", 100)]
    srv.start()
    assert srv.wait_all(100, timeout=60)
    srv.stop()
    assert [k for _, k in srv.launches] == [64, 36]
    check_results(ex, reqs)


def test_admission_by_budget(pool):
    ex = OracleExecutor(pool, delay=0.01)
    budget = ex.footprint("s10", 16)
    srv = Server(ex, hbm_budget=budget, workers=4)
    reqs = [srv.submit("s10", r) for r in roots_for(pool, "s10", 50)]
    srv.start()
    assert srv.wait_all(50, timeout=60)
    srv.stop()
    assert max(k for _, k in srv.launches) <= 16
    assert srv.max_used <= budget
    check_results(ex, reqs)


def test_request_larger_than_budget_fails_cleanly(pool):
    ex = OracleExecutor(pool)
    srv = Server(ex, hbm_budget=ex.footprint("s8", 1) - 1, workers=1)
    r = srv.submit("s8", 3)
    srv.start()
    assert srv.wait_all(1, timeout=30)
    srv.stop()
    assert r.error and "insufficient" in r.error
    assert srv.launches == []


def test_concurrency_bounded_by_workers(pool):
    ex = OracleExecutor(pool, delay=0.05)
    srv = Server(ex, hbm_budget=1 << 40, workers=3, max_batch=2).start()
    reqs = [srv.submit("s8", r) for r in roots_for(pool, "s8", 24)]
    assert srv.wait_all(24, timeout=60)
    srv.stop()
    assert 2 <= ex.max_active <= 3
    assert srv.max_inflight <= 3
    check_results(ex, reqs)


def test_oldest_head_first(pool):
    ex = OracleExecutor(pool)
    srv = Server(ex, hbm_budget=1 << 40, workers=1)
    a = roots_for(pool, "s8", 2)
    b = roots_for(pool, "s10", 2)
    srv.submit("s10", b[0])
    srv.submit("s8", a[0])
    srv.submit("s8", a[1])
    srv.submit("s10", b[1])
    srv.start()
    assert srv.wait_all(4, timeout=30)
    srv.stop()
    assert srv.launches == [("s10", 2), ("s8", 2)]


def test_range_fallback_to_single(pool):
    # levels on a 300-path exceed the limit: the batch is retried root by root
    ex = OracleExecutor(pool, range_limit=127)
    srv = Server(ex, hbm_budget=1 << 40, workers=1)
    reqs = [srv.submit("path", r) for r in (0, 150, 299)]
    srv.start()
    assert srv.wait_all(3, timeout=30)
    srv.stop()
    check_results(ex, reqs)
    assert [c for c in ex.calls if c[3]] and len([c for c in ex.calls if c[3]]) == 3


def test_continuous_batching(pool):
    # requests that arrive while a batch runs are admitted into the next launch
    ex = OracleExecutor(pool, delay=0.1)
    srv = Server(ex, hbm_budget=1 << 40, workers=1).start()
    rs = roots_for(pool, "s10", 30)
    reqs = [srv.submit("s10", rs[0])]
    time.sleep(0.03)  # first launch is running
    reqs += [srv.submit("s10", r) for r in rs[1:]]
    assert srv.wait_all(30, timeout=60)
    srv.stop()
    assert [k for _, k in srv.launches] == [1, 29]
    check_results(ex, reqs)
    assert max(r.latency for r in reqs[1:]) < 0.5


def test_executor_error_reported(pool):
    class Broken(OracleExecutor):
        def run(self, g, roots, wid, single=False):
            raise RuntimeError("device lost")
    ex = Broken(pool)
    srv = Server(ex, hbm_budget=1 << 40, workers=1).start()
    r = srv.submit("s8", 1)
    assert srv.wait_all(1, timeout=30)
    srv.stop()
    assert r.error and "device lost" in r.error
