"""Seeded synthetic Kronecker inputs shared by the oracle and the GPU path.

This module generates inputs only: edge tuples, the set of vertices that have
at least one non-loop edge, and roots drawn from that set.  It contains no part
of graph construction or breadth-first search.  The generator definition (the
initiator (A, B, C, D) = (0.57, 0.19, 0.19, 0.05), SplitMix64 counters and the
relabel bijection) is documented in ``kron_core.h``.

Sizes follow Section 2.1 of the paper: n = 2^scale vertices and
m = edgefactor * n generated tuples.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
_host = None
_dev = None

GRAPH_SEED_BASE = 1000   # graph seed = 1000 + scale
ROOT_SEED_BASE = 2000    # root seed  = 2000 + scale
MASK64 = (1 << 64) - 1
GAMMA = 0x9E3779B97F4A7C15


def _load_host():
    global _host
    if _host is None:
        path = os.path.join(HERE, "libkron_host.so")
        if not os.path.exists(path):
            raise RuntimeError(f"{path} is missing: run __graft_entry__.build() first")
        lib = ctypes.CDLL(path)
        lib.kron_edges_host.argtypes = [ctypes.c_int, ctypes.c_uint64, ctypes.c_int,
                                        ctypes.c_int64, ctypes.c_int64, ctypes.c_void_p]
        lib.kron_edges_host.restype = ctypes.c_int
        lib.kron_relabel_host.argtypes = [ctypes.c_int, ctypes.c_uint64, ctypes.c_void_p,
                                          ctypes.c_int64, ctypes.c_void_p]
        lib.kron_relabel_host.restype = ctypes.c_int
        lib.kron_nonisolated_host.argtypes = [ctypes.c_void_p, ctypes.c_int64,
                                              ctypes.c_int64, ctypes.c_void_p]
        lib.kron_nonisolated_host.restype = ctypes.c_int
        lib.kron_weights_host.argtypes = [ctypes.c_uint64, ctypes.c_int64, ctypes.c_int64,
                                          ctypes.c_void_p]
        lib.kron_weights_host.restype = ctypes.c_int
        lib.kron_splitmix64_at.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
        lib.kron_splitmix64_at.restype = ctypes.c_uint64
        _host = lib
    return _host


def _load_dev():
    global _dev
    if _dev is None:
        import torch  # noqa: F401  (bind to torch's HIP runtime; see the g5 binding)
        path = os.path.join(HERE, "libkron_dev.so")
        if not os.path.exists(path):
            raise RuntimeError(f"{path} is missing: run __graft_entry__.build() first")
        lib = ctypes.CDLL(path)
        lib.kron_edges_device.argtypes = [ctypes.c_int, ctypes.c_uint64, ctypes.c_int,
                                          ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p]
        lib.kron_edges_device.restype = ctypes.c_int
        lib.kron_nonisolated_device.argtypes = [ctypes.c_void_p, ctypes.c_int64,
                                                ctypes.c_int64, ctypes.c_void_p,
                                                ctypes.c_void_p, ctypes.c_void_p]
        lib.kron_nonisolated_device.restype = ctypes.c_int
        lib.kron_weights_device.argtypes = [ctypes.c_uint64, ctypes.c_int64, ctypes.c_void_p,
                                            ctypes.c_void_p]
        lib.kron_weights_device.restype = ctypes.c_int
        _dev = lib
    return _dev


def graph_seed(scale):
    return GRAPH_SEED_BASE + scale


def root_seed(scale):
    return ROOT_SEED_BASE + scale


def num_tuples(scale, edgefactor=16):
    return edgefactor * (1 << scale)


def splitmix64_at(state, c):
    """c-th output of SplitMix64 started at ``state`` (Steele et al. 2014)."""
    z = (state + (c + 1) * GAMMA) & MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return z ^ (z >> 31)


def edges_host(scale, edgefactor=16, seed=None, relabel=True, start=0, stop=None):
    """Tuples [start, stop) as an int64 numpy array of shape [stop-start, 2]."""
    if seed is None:
        seed = graph_seed(scale)
    m = num_tuples(scale, edgefactor)
    stop = m if stop is None else stop
    out = np.empty((stop - start, 2), dtype=np.int64)
    rc = _load_host().kron_edges_host(scale, seed, int(bool(relabel)), start, stop,
                                      out.ctypes.data)
    if rc != 0:
        raise ValueError(f"kron_edges_host rejected scale={scale} range=[{start},{stop})")
    return out


def relabel_host(scale, seed, x):
    x = np.ascontiguousarray(x, dtype=np.int64)
    out = np.empty_like(x)
    if _load_host().kron_relabel_host(scale, seed, x.ctypes.data, x.size, out.ctypes.data):
        raise ValueError("bad scale")
    return out


def edges_device(scale, edgefactor=16, seed=None, relabel=True, device="cuda"):
    """The same tuples as :func:`edges_host`, generated straight into HBM."""
    import torch
    if seed is None:
        seed = graph_seed(scale)
    m = num_tuples(scale, edgefactor)
    out = torch.empty((m, 2), dtype=torch.int64, device=device)
    stream = torch.cuda.current_stream(out.device).cuda_stream
    rc = _load_dev().kron_edges_device(scale, seed, int(bool(relabel)), m, out.data_ptr(),
                                       stream)
    if rc != 0:
        raise RuntimeError(f"kron_edges_device failed ({rc})")
    return out


def weights_host(scale, edgefactor=16, seed=None, start=0, stop=None):
    """Integer weights in [1, 255] of tuples [start, stop) as a uint8 numpy
    array (the weight row of the paper's 3 x #E tuple matrix)."""
    if seed is None:
        seed = graph_seed(scale)
    m = num_tuples(scale, edgefactor)
    stop = m if stop is None else stop
    out = np.empty(stop - start, dtype=np.uint8)
    if _load_host().kron_weights_host(seed, start, stop, out.ctypes.data) != 0:
        raise ValueError("bad tuple range")
    return out


def weights_device(scale, edgefactor=16, seed=None, device="cuda"):
    """The same weights as :func:`weights_host`, generated straight into HBM."""
    import torch
    if seed is None:
        seed = graph_seed(scale)
    m = num_tuples(scale, edgefactor)
    out = torch.empty(m, dtype=torch.uint8, device=device)
    stream = torch.cuda.current_stream(out.device).cuda_stream
    if _load_dev().kron_weights_device(seed, m, out.data_ptr(), stream) != 0:
        raise RuntimeError("kron_weights_device failed")
    return out


def nonisolated_host(edges, n):
    """uint8 mask: 1 where the vertex ends some non-loop tuple."""
    edges = np.ascontiguousarray(edges, dtype=np.int64)
    mask = np.empty(n, dtype=np.uint8)
    if _load_host().kron_nonisolated_host(edges.ctypes.data, edges.shape[0], n,
                                          mask.ctypes.data):
        raise ValueError("edge id outside [0, n)")
    return mask


def nonisolated_device(edges, n):
    import torch
    mask = torch.empty(n, dtype=torch.uint8, device=edges.device)
    bad = torch.zeros(1, dtype=torch.int32, device=edges.device)
    stream = torch.cuda.current_stream(edges.device).cuda_stream
    rc = _load_dev().kron_nonisolated_device(edges.data_ptr(), edges.shape[0], n,
                                             mask.data_ptr(), bad.data_ptr(), stream)
    if rc != 0 or int(bad.item()) != 0:
        raise RuntimeError("kron_nonisolated_device failed")
    return mask


def select_roots(mask, k, seed):
    """k distinct roots drawn uniformly from {v : mask[v] != 0}.

    Candidate t is splitmix64_at(splitmix64_at(seed, 2), t) mod n; candidates
    with mask 0 or already chosen are rejected.  ``mask`` is a numpy array (or
    anything np.asarray accepts) of length n.
    """
    mask = np.asarray(mask)
    n = mask.shape[0]
    avail = int(np.count_nonzero(mask))
    if k > avail:
        raise ValueError(f"only {avail} vertices have degree >= 1; asked for {k} roots")
    base = splitmix64_at(seed, 2)
    roots, seen, t = [], set(), 0
    while len(roots) < k:
        c = splitmix64_at(base, t) % n
        t += 1
        if mask[c] and c not in seen:
            seen.add(c)
            roots.append(int(c))
    return roots
