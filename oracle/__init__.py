"""CPU oracle for CSR construction and breadth-first search.

TEST INFRASTRUCTURE ONLY: imported by tests/, __graft_entry__.smoke() and the
cpu_baseline leg of bench.py, never by the GPU library (the two share no code).

Python bindings (numpy in, numpy out) for ``oracle.c``:

* :func:`build_csr` -- Kernel 1 (Section 2.2): undirected CSR, self-loops and
  repeated edges dropped, rows ascending, empty rows repeat the previous index.
* :func:`bfs` -- Kernel 2 (Section 2.3.1, "Sequential BFS"): queue BFS with
  visited marked at discovery; parent[root] = root; -1 for unreached.
* :func:`bfs_batch` -- the single-root BFS per root, levels cast to int8.
* :func:`components`, :func:`validate`, :func:`validate_edges` -- independent
  checks of a BFS result (union-find reached set, tree edges, level rules);
  :func:`check_parents` -- the parent rules alone, for levels already compared
  bit-exactly with :func:`bfs`.
* :func:`teps_edges` -- m_r, the distinct undirected edges of the root's
  component (traversed edges for TEPS, Section 4.3).
* :func:`min_parents` -- the deterministic parent choice: the smallest-id
  neighbour one level up.
* :func:`build_csr_w`, :func:`sssp`, :func:`check_sssp`, :func:`min_prev` --
  Kernel 3 (Section 2.4, "Sequential SSSP"): the weighted CSR (smallest weight
  of repeated tuples), Dijkstra's distances and predecessors, an independent
  validator, and the deterministic predecessor choice.
"""
import ctypes
import os
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
_lib = None

RULES = {
    0: "valid",
    1: "root is not its own parent or not at level 0",
    2: "value out of range or parent/level reached-ness disagree",
    3: "tree edge is not a graph edge",
    4: "parent level is not child level - 1",
    5: "reached set is not the root's connected component",
    6: "an edge spans more than one level",
    7: "a vertex other than the root has level 0",
}


def _load():
    global _lib
    if _lib is None:
        path = os.path.join(HERE, "liboracle.so")
        if not os.path.exists(path):
            raise RuntimeError(f"{path} is missing: run __graft_entry__.build() first")
        lib = ctypes.CDLL(path)
        P = ctypes.c_void_p
        I64 = ctypes.c_int64
        lib.orc_build_csr.argtypes = [P, I64, I64, P, P]
        lib.orc_build_csr.restype = I64
        lib.orc_bfs.argtypes = [P, P, I64, I64, P, P]
        lib.orc_bfs.restype = I64
        lib.orc_components.argtypes = [P, I64, I64, P]
        lib.orc_components.restype = I64
        lib.orc_validate.argtypes = [P, P, I64, I64, P, P, P]
        lib.orc_validate.restype = ctypes.c_int
        lib.orc_validate_edges.argtypes = [P, I64, I64, I64, P, P]
        lib.orc_validate_edges.restype = ctypes.c_int
        lib.orc_build_csr_w.argtypes = [P, P, I64, I64, P, P, P]
        lib.orc_build_csr_w.restype = I64
        lib.orc_sssp.argtypes = [P, P, P, I64, I64, P, P]
        lib.orc_sssp.restype = I64
        lib.orc_check_sssp.argtypes = [P, P, P, I64, I64, P, P]
        lib.orc_check_sssp.restype = ctypes.c_int
        lib.orc_min_prev.argtypes = [P, P, P, I64, I64, P, P]
        lib.orc_min_prev.restype = ctypes.c_int
        lib.orc_check_parents.argtypes = [P, P, I64, I64, P, P]
        lib.orc_check_parents.restype = ctypes.c_int
        lib.orc_teps_edges.argtypes = [P, I64, P]
        lib.orc_teps_edges.restype = I64
        lib.orc_min_parents.argtypes = [P, P, I64, I64, P, P]
        lib.orc_min_parents.restype = ctypes.c_int
        _lib = lib
    return _lib


def _edges(edges):
    e = np.ascontiguousarray(edges, dtype=np.int64)
    if e.ndim != 2 or e.shape[1] != 2:
        e = e.reshape(-1, 2)
    return e


class Csr:
    """Oracle CSR: row_ptr int64[n+1], col_idx int32[nnz]."""

    def __init__(self, row_ptr, col_idx):
        self.row_ptr = row_ptr
        self.col_idx = col_idx
        self.n = row_ptr.shape[0] - 1
        self.nnz = int(row_ptr[-1])

    def degree(self):
        return np.diff(self.row_ptr)

    def row(self, v):
        return self.col_idx[self.row_ptr[v]:self.row_ptr[v + 1]]


def build_csr(edges, n):
    e = _edges(edges)
    m = e.shape[0]
    rp = np.empty(n + 1, dtype=np.int64)
    ci = np.empty(max(2 * m, 1), dtype=np.int32)
    nnz = _load().orc_build_csr(e.ctypes.data, m, n, rp.ctypes.data, ci.ctypes.data)
    if nnz < 0:
        raise ValueError(f"orc_build_csr failed ({nnz}): vertex id outside [0, {n})"
                         if nnz == -1 else f"orc_build_csr failed ({nnz})")
    return Csr(rp, ci[:nnz].copy())


def bfs(csr, root):
    """(parent int32[n], level int32[n]) from root."""
    n = csr.n
    parent = np.empty(n, dtype=np.int32)
    level = np.empty(n, dtype=np.int32)
    ci = csr.col_idx if csr.col_idx.size else np.zeros(1, np.int32)
    r = _load().orc_bfs(csr.row_ptr.ctypes.data, ci.ctypes.data, n, int(root),
                        parent.ctypes.data, level.ctypes.data)
    if r < 0:
        raise ValueError(f"orc_bfs failed ({r}) for root {root}")
    return parent, level


def bfs_timed(csr, root):
    """bfs() plus the wall time of the traversal alone (seconds)."""
    n = csr.n
    parent = np.empty(n, dtype=np.int32)
    level = np.empty(n, dtype=np.int32)
    ci = csr.col_idx if csr.col_idx.size else np.zeros(1, np.int32)
    lib = _load()
    t0 = time.perf_counter()
    r = lib.orc_bfs(csr.row_ptr.ctypes.data, ci.ctypes.data, n, int(root),
                    parent.ctypes.data, level.ctypes.data)
    t1 = time.perf_counter()
    if r < 0:
        raise ValueError(f"orc_bfs failed ({r}) for root {root}")
    return parent, level, t1 - t0


def bfs_batch(csr, roots):
    """(parents int32[k][n], levels int8[k][n]): single-root BFS per root."""
    k = len(roots)
    parents = np.empty((k, csr.n), dtype=np.int32)
    levels = np.empty((k, csr.n), dtype=np.int8)
    for i, r in enumerate(roots):
        p, lv = bfs(csr, r)
        if lv.max(initial=0) > 127:
            raise ValueError("level exceeds int8")
        parents[i] = p
        levels[i] = lv.astype(np.int8)
    return parents, levels


def components(edges, n):
    e = _edges(edges)
    label = np.empty(n, dtype=np.int64)
    c = _load().orc_components(e.ctypes.data, e.shape[0], n, label.ctypes.data)
    if c < 0:
        raise ValueError("orc_components failed")
    return label


def validate(csr, root, parent, level, label):
    """0 if (parent, level) is a valid BFS result from root, else a rule number."""
    parent = np.ascontiguousarray(parent, dtype=np.int32)
    level = np.ascontiguousarray(level, dtype=np.int32)
    label = np.ascontiguousarray(label, dtype=np.int64)
    ci = csr.col_idx if csr.col_idx.size else np.zeros(1, np.int32)
    return _load().orc_validate(csr.row_ptr.ctypes.data, ci.ctypes.data, csr.n, int(root),
                                parent.ctypes.data, level.ctypes.data, label.ctypes.data)


def validate_edges(edges, n, root, parent, level):
    """validate() from the tuple list alone (no CSR, no union-find)."""
    e = _edges(edges)
    parent = np.ascontiguousarray(parent, dtype=np.int32)
    level = np.ascontiguousarray(level, dtype=np.int32)
    return _load().orc_validate_edges(e.ctypes.data, e.shape[0], n, int(root),
                                      parent.ctypes.data, level.ctypes.data)


def check_parents(csr, root, parent, level):
    """Parent rules of validate() for a level array known to be exact; 0 or a
    rule number.  Parallel over vertices, so it suits full-size graphs."""
    parent = np.ascontiguousarray(parent, dtype=np.int32)
    level = np.ascontiguousarray(level, dtype=np.int32)
    ci = csr.col_idx if csr.col_idx.size else np.zeros(1, np.int32)
    return _load().orc_check_parents(csr.row_ptr.ctypes.data, ci.ctypes.data, csr.n, int(root),
                                     parent.ctypes.data, level.ctypes.data)


def teps_edges(csr, level):
    level = np.ascontiguousarray(level, dtype=np.int32)
    return int(_load().orc_teps_edges(csr.row_ptr.ctypes.data, csr.n, level.ctypes.data))


def min_parents(csr, root, level):
    """parent[v] = smallest-id neighbour of v at level[v] - 1 (root: itself)."""
    level = np.ascontiguousarray(level, dtype=np.int32)
    parent = np.empty(csr.n, dtype=np.int32)
    ci = csr.col_idx if csr.col_idx.size else np.zeros(1, np.int32)
    rc = _load().orc_min_parents(csr.row_ptr.ctypes.data, ci.ctypes.data, csr.n, int(root),
                                 level.ctypes.data, parent.ctypes.data)
    if rc != 0:
        raise ValueError("a reached vertex has no neighbour one level up")
    return parent


INF32 = 0xFFFFFFFF

SSSP_RULES = {
    0: "valid",
    1: "dist[src] != 0 or prev[src] != src",
    2: "value out of range, or infinity and prev = -1 disagree",
    3: "prev[v] is not a neighbour of v",
    4: "dist[v] != dist[prev[v]] + w(prev[v], v)",
    5: "an edge can shorten a distance (or joins reached and unreached)",
    6: "prev pointers of a reached vertex do not lead back to the source",
}


class CsrW(Csr):
    """Weighted oracle CSR: row_ptr, col_idx and weights uint8[nnz]."""

    def __init__(self, row_ptr, col_idx, weights):
        super().__init__(row_ptr, col_idx)
        self.weights = weights

    def row_weights(self, v):
        return self.weights[self.row_ptr[v]:self.row_ptr[v + 1]]


def build_csr_w(edges, weights, n):
    e = _edges(edges)
    w = np.ascontiguousarray(weights, dtype=np.uint8)
    if w.shape[0] != e.shape[0]:
        raise ValueError("one weight per tuple")
    m = e.shape[0]
    rp = np.empty(n + 1, dtype=np.int64)
    ci = np.empty(max(2 * m, 1), dtype=np.int32)
    wt = np.empty(max(2 * m, 1), dtype=np.uint8)
    nnz = _load().orc_build_csr_w(e.ctypes.data, w.ctypes.data, m, n, rp.ctypes.data,
                                  ci.ctypes.data, wt.ctypes.data)
    if nnz < 0:
        raise ValueError(f"orc_build_csr_w failed ({nnz})")
    return CsrW(rp, ci[:nnz].copy(), wt[:nnz].copy())


def _wargs(csr):
    ci = csr.col_idx if csr.col_idx.size else np.zeros(1, np.int32)
    wt = csr.weights if csr.weights.size else np.zeros(1, np.uint8)
    return csr.row_ptr.ctypes.data, ci.ctypes.data, wt.ctypes.data, ci, wt


def sssp(csr, src):
    """(dist uint32[n], prev int32[n]) by Dijkstra; INF32 / -1 when unreached."""
    rp, ci, wt, _k1, _k2 = _wargs(csr)
    dist = np.empty(csr.n, dtype=np.uint32)
    prev = np.empty(csr.n, dtype=np.int32)
    r = _load().orc_sssp(rp, ci, wt, csr.n, int(src), dist.ctypes.data, prev.ctypes.data)
    if r < 0:
        raise ValueError(f"orc_sssp failed ({r}) for source {src}")
    return dist, prev


def sssp_timed(csr, src):
    """sssp() plus the wall time of the Dijkstra call alone (seconds)."""
    rp, ci, wt, _k1, _k2 = _wargs(csr)
    dist = np.empty(csr.n, dtype=np.uint32)
    prev = np.empty(csr.n, dtype=np.int32)
    lib = _load()
    t0 = time.perf_counter()
    r = lib.orc_sssp(rp, ci, wt, csr.n, int(src), dist.ctypes.data, prev.ctypes.data)
    t1 = time.perf_counter()
    if r < 0:
        raise ValueError(f"orc_sssp failed ({r}) for source {src}")
    return dist, prev, t1 - t0


def check_sssp(csr, src, dist, prev):
    """0 if (dist, prev) is an exact shortest-path result from src, else a rule."""
    rp, ci, wt, _k1, _k2 = _wargs(csr)
    dist = np.ascontiguousarray(dist, dtype=np.uint32)
    prev = np.ascontiguousarray(prev, dtype=np.int32)
    return _load().orc_check_sssp(rp, ci, wt, csr.n, int(src), dist.ctypes.data,
                                  prev.ctypes.data)


def min_prev(csr, src, dist):
    """prev[v] = smallest-id neighbour u with dist[u] + w(u, v) = dist[v]."""
    rp, ci, wt, _k1, _k2 = _wargs(csr)
    dist = np.ascontiguousarray(dist, dtype=np.uint32)
    prev = np.empty(csr.n, dtype=np.int32)
    if _load().orc_min_prev(rp, ci, wt, csr.n, int(src), dist.ctypes.data, prev.ctypes.data):
        raise ValueError("a reached vertex has no tight neighbour")
    return prev
