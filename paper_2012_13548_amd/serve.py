"""Continuous-batching BFS serving over a pool of resident graphs (one GPU).

Requests (graph, root) arrive at any time.  A dispatcher thread keeps one
pending queue per graph and, whenever a worker is free and the HBM budget
allows, launches the oldest graph's pending requests together (up to 64 roots)
as one batched BFS on that worker's stream; requests that arrive while other
batches run join the next launch.  Work of different workers overlaps on the
device.  Results stay on the device (rows of the batch's level/parent tensors).

The executor does the traversal: :class:`GpuExecutor` calls g5_bfs_batch in
stepped mode (one plain launch per level, safe next to other streams) or g5_bfs
for a lone request; tests drive the scheduler with a CPU executor.

CLI (on a machine with the GPU): ``python -m paper_2012_13548_amd.serve --scales 16 18 20
22 23 --requests 10000`` prints one JSON line with p50/p99 latency and
aggregate TEPS under a Poisson arrival stream.
"""
import argparse
import collections
import json
import threading
import time

import numpy as np

MAX_BATCH = 64


class RangeExceeded(Exception):
    """A batched level does not fit int8; the requests are retried one by one."""


class Request:
    __slots__ = ("rid", "graph", "root", "t_arrival", "t_start", "t_done", "parent", "level",
                 "error", "m_r", "batch_id", "batch_size")

    def __init__(self, rid, graph, root, t_arrival):
        self.rid, self.graph, self.root, self.t_arrival = rid, graph, root, t_arrival
        self.t_start = self.t_done = None
        self.parent = self.level = self.error = None
        self.m_r = None
        self.batch_id = self.batch_size = None

    @property
    def latency(self):
        return None if self.t_done is None else self.t_done - self.t_arrival


class Server:
    """Scheduler: per-graph queues, oldest-head-first dispatch, HBM admission.

    executor must provide ``graphs`` (name -> vertex count), ``footprint(graph,
    k)`` (device bytes one launch of k roots needs while it runs) and
    ``run(graph, roots, worker) -> (parents [k][n] or None, levels [k][n])``,
    returning once the results are complete; ``run`` raises
    :class:`RangeExceeded` when a batched level does not fit.  An optional
    ``edges(graph, level_rows, worker) -> list`` gives each request's traversed
    edges m_r; it is called after the request's completion time is taken, so
    the bookkeeping is not part of its latency.
    """

    def __init__(self, executor, hbm_budget, workers=4, max_batch=MAX_BATCH,
                 clock=time.monotonic, keep_results=True):
        self.ex = executor
        self.budget = int(hbm_budget)
        self.free = int(hbm_budget)
        self.max_batch = max(1, min(max_batch, MAX_BATCH))
        self.nworkers = workers
        self.clock = clock
        self.keep = keep_results
        self.cv = threading.Condition()
        self.pending = {g: collections.deque() for g in executor.graphs}
        self.jobs = collections.deque()
        self.inflight = 0
        self.max_inflight = 0
        self.max_used = 0
        self.done = []
        self.launches = []       # (graph, k) per launch
        self.stopping = False
        self.next_rid = 0
        self.threads = []

    # ------------------------------------------------------------ client side
    def submit(self, graph, root):
        with self.cv:
            if graph not in self.pending:
                raise KeyError(f"unknown graph {graph!r}")
            r = Request(self.next_rid, graph, int(root), self.clock())
            self.next_rid += 1
            self.pending[graph].append(r)
            self.cv.notify_all()
            return r

    def start(self):
        self.threads = [threading.Thread(target=self._dispatch, name="g5-dispatch", daemon=True)]
        self.threads += [threading.Thread(target=self._work, args=(i,), name=f"g5-worker{i}",
                                          daemon=True) for i in range(self.nworkers)]
        for t in self.threads:
            t.start()
        return self

    def stop(self, timeout=None):
        """Drain every submitted request, then stop the threads."""
        with self.cv:
            self.stopping = True
            self.cv.notify_all()
        for t in self.threads:
            t.join(timeout)

    def wait_all(self, n, timeout=None):
        t_end = None if timeout is None else time.monotonic() + timeout
        with self.cv:
            while len(self.done) < n:
                left = None if t_end is None else t_end - time.monotonic()
                if left is not None and left <= 0:
                    return False
                self.cv.wait(left)
        return True

    # ------------------------------------------------------------ scheduler
    def _pick(self):
        """Oldest pending head across graphs, sized to fit the free budget."""
        heads = [(q[0].t_arrival, q[0].rid, g) for g, q in self.pending.items() if q]
        if not heads:
            return None
        _, _, g = min(heads)
        q = self.pending[g]
        k = min(len(q), self.max_batch)
        while k >= 1 and self.ex.footprint(g, k) > self.free:
            k //= 2
        if k == 0:
            if self.ex.footprint(g, 1) > self.budget:
                r = q.popleft()
                r.error = "insufficient HBM budget for one request"
                r.t_done = self.clock()
                self.done.append(r)
                self.cv.notify_all()
                return "progress"
            return None
        reqs = [q.popleft() for _ in range(k)]
        fp = self.ex.footprint(g, k)
        return g, reqs, fp

    def _dispatch(self):
        with self.cv:
            while True:
                busy = self.inflight >= self.nworkers
                job = None if busy else self._pick()
                if job == "progress":
                    continue
                if job is not None:
                    g, reqs, fp = job
                    self.free -= fp
                    self.inflight += 1
                    self.max_inflight = max(self.max_inflight, self.inflight)
                    self.max_used = max(self.max_used, self.budget - self.free)
                    self.jobs.append(job)
                    self.launches.append((g, len(reqs)))
                    self.cv.notify_all()
                    continue
                if self.stopping and self.inflight == 0 and not any(self.pending.values()):
                    self.jobs.extend([None] * self.nworkers)
                    self.cv.notify_all()
                    return
                self.cv.wait()

    def _work(self, wid):
        while True:
            with self.cv:
                while not self.jobs:
                    self.cv.wait()
                job = self.jobs.popleft()
            if job is None:
                return
            g, reqs, fp = job
            t0 = self.clock()
            for r in reqs:
                r.t_start = t0
                r.batch_size = len(reqs)
            rows = None
            try:
                rows = self._run(g, reqs, wid)
            except Exception as e:  # noqa: BLE001 - reported per request
                for r in reqs:
                    r.error = f"{type(e).__name__}: {e}"
            t1 = self.clock()
            # TEPS bookkeeping after the completion time: not part of latency
            if rows is not None and hasattr(self.ex, "edges"):
                try:
                    for r, mr in zip(reqs, self.ex.edges(g, [lv for _, lv in rows], wid)):
                        r.m_r = mr
                except Exception as e:  # noqa: BLE001 - reported per request
                    for r in reqs:
                        r.error = f"{type(e).__name__}: {e}"
            with self.cv:
                for r in reqs:
                    r.t_done = t1
                    self.done.append(r)
                self.free += fp
                self.inflight -= 1
                self.cv.notify_all()

    def _run(self, g, reqs, wid):
        """Runs the launch; returns one (parent, level) row per request."""
        roots = [r.root for r in reqs]
        try:
            parents, levels = self.ex.run(g, roots, wid)
            rows = [(None if parents is None else parents[i], levels[i])
                    for i in range(len(reqs))]
        except RangeExceeded:
            rows = []
            for root in roots:
                p, lv = self.ex.run(g, [root], wid, single=True)
                rows.append((None if p is None else p[0], lv[0]))
        for r, (p, lv) in zip(reqs, rows):
            if self.keep:
                r.parent, r.level = p, lv
        return rows

    # ------------------------------------------------------------ statistics
    def summary(self, t_first=None, t_last=None):
        ok = [r for r in self.done if r.error is None]
        lat = np.array([r.latency for r in ok]) * 1e3 if ok else np.zeros(1)
        t0 = min(r.t_arrival for r in self.done) if t_first is None else t_first
        t1 = max(r.t_done for r in self.done) if t_last is None else t_last
        edges = sum(r.m_r for r in ok if r.m_r is not None)
        sizes = [k for _, k in self.launches]
        kinds = {}
        for r in self.done:
            if r.error is not None:
                kinds[r.error] = kinds.get(r.error, 0) + 1
        return {"requests": len(self.done), "errors": len(self.done) - len(ok),
                "error_kinds": dict(sorted(kinds.items(), key=lambda kv: -kv[1])[:3]),
                "p50_ms": round(float(np.percentile(lat, 50)), 3),
                "p99_ms": round(float(np.percentile(lat, 99)), 3),
                "mean_ms": round(float(lat.mean()), 3),
                "wall_s": round(t1 - t0, 3),
                "throughput_rps": round(len(ok) / max(t1 - t0, 1e-9), 1),
                "aggregate_gteps": round(edges / max(t1 - t0, 1e-9) / 1e9, 3),
                "launches": len(sizes), "mean_batch": round(float(np.mean(sizes)), 2) if sizes else 0,
                "max_inflight": self.max_inflight, "max_hbm_used": self.max_used}


class GpuExecutor:
    """Runs batches through the g5 C-ABI on one stream per worker.

    graphs: name -> Csr.  A launch of k roots holds levels (k*n int8), parents
    (k*n int32) and the batch masks (4 * 8n bytes) while it runs.
    """

    def __init__(self, csrs, workers, parents=True, count_edges=True):
        import torch
        import paper_2012_13548_amd as g5
        self.g5, self.torch = g5, torch
        self.csrs = csrs
        self.graphs = {k: c.n for k, c in csrs.items()}
        self.parents = parents
        self.streams = [torch.cuda.Stream(device=c.device) for c in
                        [next(iter(csrs.values()))] * workers]
        self.deg = {}
        if count_edges:
            for k, c in csrs.items():
                rp, _ = c.arrays()
                self.deg[k] = (rp[1:] - rp[:-1]).to(torch.int64)

    def footprint(self, graph, k):
        n = self.graphs[graph]
        out = k * n * (5 if self.parents else 1)
        return out + (32 * n if k > 1 else 8 * n)

    def run(self, graph, roots, wid, single=False):
        torch, g5 = self.torch, self.g5
        csr = self.csrs[graph]
        with torch.cuda.stream(self.streams[wid]):
            if len(roots) == 1:
                p, lv = g5.bfs(csr, roots[0])
                parents, levels = (p[None] if self.parents else None), lv[None]
            else:
                try:
                    parents, levels = g5.bfs_batch(csr, roots, parents=self.parents, stepped=True)
                except g5.G5Error as e:
                    if e.status == g5.G5_ERANGE:
                        raise RangeExceeded(str(e)) from e
                    raise
            self.streams[wid].synchronize()
        return parents, levels

    def edges(self, graph, level_rows, wid):
        """m_r of each level row: half the degree sum of its reached vertices,
        reduced on the device in groups of rows and read back once."""
        torch = self.torch
        if graph not in self.deg:
            return [None] * len(level_rows)
        deg = self.deg[graph]
        with torch.cuda.stream(self.streams[wid]):
            sums = []
            for i in range(0, len(level_rows), 8):
                lv = torch.stack(level_rows[i:i + 8])
                sums.append(((lv >= 0).to(deg.dtype) * deg[None, :]).sum(dim=1))
            out = (torch.cat(sums) // 2).tolist()
        return out


def poisson_run(server, graphs, roots_of, rate, count, seed=3000, t_limit=None):
    """Submit `count` requests with exponential gaps (rate per second), graph
    uniform over `graphs`, root uniform over roots_of[graph]; returns the
    requests in submission order."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, size=count)
    picks = rng.integers(0, len(graphs), size=count)
    reqs = []
    t_next = time.monotonic()
    for i in range(count):
        t_next += gaps[i]
        d = t_next - time.monotonic()
        if d > 0:
            time.sleep(d)
        g = graphs[picks[i]]
        cand = roots_of[g]
        reqs.append(server.submit(g, int(cand[rng.integers(0, len(cand))])))
        if t_limit is not None and time.monotonic() > t_limit:
            break
    return reqs


def run_poisson(scales=(16, 18, 20, 22, 23), requests=10000, workers=4, load=0.7,
                budget_gb=0.0, log=None):
    """Graphs of the given scales resident at once; a calibration run (2,000
    requests queued at once) gives the saturated rate, then `requests` Poisson
    arrivals at `load` times that rate.  Returns the summary with the run's
    settings."""
    import torch
    import kronecker as K
    import paper_2012_13548_amd as g5
    log = log or (lambda msg: None)
    dev = torch.device("cuda:0")
    csrs, roots_of = {}, {}
    for s in scales:
        e = K.edges_device(s, device=dev)
        name = f"s{s}"
        csrs[name] = g5.build_csr(e, 1 << s)
        mask = K.nonisolated_device(e, 1 << s).cpu().numpy()
        roots_of[name] = np.flatnonzero(mask)
        del e
        torch.cuda.empty_cache()
        log(f"graph {name}: nnz {csrs[name].nnz}")
    names = list(csrs)
    free, _ = torch.cuda.mem_get_info()
    budget = int(budget_gb * 2**30) if budget_gb > 0 else int(0.8 * free)
    ex = GpuExecutor(csrs, workers)
    # warm-up: every graph once
    for gname in names:
        ex.run(gname, list(roots_of[gname][:2]), 0)
    # calibration: saturated throughput with everything queued at once
    cal = Server(ex, budget, workers=workers, keep_results=False).start()
    ncal = min(2000, requests)
    rng = np.random.default_rng(1)
    t0 = time.monotonic()
    for i in range(ncal):
        gname = names[i % len(names)]
        cal.submit(gname, int(roots_of[gname][rng.integers(0, len(roots_of[gname]))]))
    cal.wait_all(ncal)
    sat = ncal / (time.monotonic() - t0)
    cal.stop()
    rate = load * sat
    log(f"saturated {sat:.1f} req/s -> Poisson rate {rate:.1f} req/s")
    srv = Server(ex, budget, workers=workers, keep_results=False).start()
    t_start = time.monotonic()
    reqs = poisson_run(srv, names, roots_of, rate, requests)
    srv.wait_all(len(reqs))
    srv.stop()
    out = srv.summary(t_first=t_start)
    out.update({"scales": list(scales), "workers": workers, "rate_rps": round(rate, 1),
                "saturated_rps": round(sat, 1), "load": load,
                "budget_gb": round(budget / 2**30, 2)})
    del ex, csrs
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser(description="Poisson serving run over resident Kronecker graphs")
    ap.add_argument("--scales", type=int, nargs="+", default=[16, 18, 20, 22, 23])
    ap.add_argument("--requests", type=int, default=10000)
    ap.add_argument("--workers", type=int, default=4)
    ap.add_argument("--load", type=float, default=0.7, help="arrival rate / saturated rate")
    ap.add_argument("--budget-gb", type=float, default=0.0, help="HBM budget (0: 80%% of free)")
    args = ap.parse_args()
    import sys

    def log(msg):
        sys.stderr.write(f"[serve] {msg}\n")
        sys.stderr.flush()

    out = run_poisson(args.scales, args.requests, args.workers, args.load, args.budget_gb, log)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
