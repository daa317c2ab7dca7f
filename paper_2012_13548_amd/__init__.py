"""g5: breadth-first search over Kronecker graphs on one MI355X (gfx950).

Thin ctypes binding of ``libg5.so`` (C-ABI declared in ``include/g5.h``).  Every
step of graph construction and traversal runs in the library's HIP kernels;
this module only marshals arguments.  PyTorch supplies device memory and the
current stream.  The library must be built (``__graft_entry__.build()``); the
import fails if it is missing.

* :func:`build_csr` -- Kernel 1 of the paper (Section 2.2): undirected CSR.
* :func:`bfs` -- Kernel 2 (Section 2.3): parent and level arrays from a root.
* :func:`bfs_batch` -- up to 64 roots in one launch.
* :func:`build_csr_w`, :func:`sssp` -- Kernel 3 (Section 2.4): weighted CSR
  and single-source shortest paths by delta-stepping.
"""
import ctypes
import os

__all__ = ["G5Error", "Csr", "build_csr", "build_csr_w", "bfs", "bfs_batch", "sssp",
           "level_work", "LIB_PATH", "lib",
           "DIR_AUTO", "DIR_TOPDOWN", "DIR_BOTTOMUP", "CLAIM_OR", "CLAIM_CAS"]

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libg5.so")

G5_OK, G5_EINVAL, G5_ENOMEM, G5_EDEVICE, G5_ERANGE = 0, -1, -2, -3, -4
STATUS = {G5_EINVAL: "G5_EINVAL", G5_ENOMEM: "G5_ENOMEM", G5_EDEVICE: "G5_EDEVICE",
          G5_ERANGE: "G5_ERANGE"}
DIR_AUTO, DIR_TOPDOWN, DIR_BOTTOMUP = 0, 1, 2
CLAIM_OR, CLAIM_CAS = 0, 1
MAX_STAT_LEVELS = 64

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                      "(there is no fallback implementation)")

# torch ships its own libamdhip64.so.7.  Loading it first makes libg5 bind to
# that same HIP runtime, so torch's device memory and streams are valid in the
# library; loading libg5 first would start a second runtime in the process.
import torch  # noqa: E402,F401

lib = ctypes.CDLL(LIB_PATH)


FLAG_TIME_STEPS, FLAG_COUNT_BYTES, FLAG_NO_HINT, FLAG_STEPPED, FLAG_PACKED = 1, 2, 4, 8, 16
FLAG_MIN_PARENT, FLAG_NO_LDS, FLAG_ROWLOOP, FLAG_PERSISTENT = 32, 64, 128, 512
FLAG_GRAPH = 1024


class BfsParams(ctypes.Structure):
    _fields_ = [("direction", ctypes.c_int32), ("bu_lane_scan", ctypes.c_int32),
                ("alpha", ctypes.c_double), ("beta", ctypes.c_double),
                ("lds_density", ctypes.c_double), ("claim", ctypes.c_int32),
                ("flags", ctypes.c_int32), ("bu_blocks_per_cu", ctypes.c_int32),
                ("lds_kb", ctypes.c_int32), ("bu_vertices_per_lane", ctypes.c_int32),
                ("td_blocks_per_cu", ctypes.c_int32), ("heavy_kedges", ctypes.c_int32),
                ("reserved", ctypes.c_int32),
                ("gamma", ctypes.c_double)]


_L = MAX_STAT_LEVELS


class BfsStats(ctypes.Structure):
    _fields_ = [("nlevels", ctypes.c_int32), ("dir", ctypes.c_int32 * _L),
                ("frontier", ctypes.c_int64 * _L), ("discovered", ctypes.c_int64 * _L),
                ("edges", ctypes.c_int64 * _L), ("bytes", ctypes.c_int64 * _L),
                ("step_ms", ctypes.c_double * _L), ("reached", ctypes.c_int64),
                ("alpha", ctypes.c_double), ("beta", ctypes.c_double),
                ("bu_lane_scan", ctypes.c_int32), ("bu_blocks_per_cu", ctypes.c_int32),
                ("lds_levels", ctypes.c_int32), ("lds_shift", ctypes.c_int32),
                ("lds_mask", ctypes.c_int64), ("heavy_mask", ctypes.c_int64),
                ("reserved", ctypes.c_int64 * 3)]


class BatchParams(ctypes.Structure):
    _fields_ = [("direction", ctypes.c_int32), ("alpha", ctypes.c_double),
                ("flags", ctypes.c_int32), ("blocks_per_cu", ctypes.c_int32),
                ("reserved", ctypes.c_int32 * 4)]


class BatchStats(ctypes.Structure):
    _fields_ = [("nlevels", ctypes.c_int32), ("dir", ctypes.c_int32 * _L),
                ("frontier", ctypes.c_int64 * _L), ("launch_ms", ctypes.c_double),
                ("grid_blocks", ctypes.c_int32), ("pad", ctypes.c_int32),
                ("alpha", ctypes.c_double), ("reserved", ctypes.c_int32 * 6)]


_P = ctypes.c_void_p
_I64 = ctypes.c_int64
_PP = ctypes.POINTER(ctypes.c_void_p)
lib.g5_build_csr.argtypes = [_P, _I64, _I64, _P, _PP]
lib.g5_build_csr.restype = ctypes.c_int
lib.g5_csr_info.argtypes = [_P, ctypes.POINTER(_I64), ctypes.POINTER(_I64), _PP, _PP]
lib.g5_csr_info.restype = ctypes.c_int
lib.g5_csr_copy.argtypes = [_P, _P, _P, _P]
lib.g5_csr_copy.restype = ctypes.c_int
lib.g5_csr_free.argtypes = [_P]
lib.g5_csr_free.restype = None
lib.g5_bfs.argtypes = [_P, _I64, _P, _P, _P]
lib.g5_bfs.restype = ctypes.c_int
lib.g5_bfs_ex.argtypes = [_P, _I64, _P, _P, _P, ctypes.POINTER(BfsParams),
                          ctypes.POINTER(BfsStats)]
lib.g5_bfs_ex.restype = ctypes.c_int
lib.g5_bfs_batch.argtypes = [_P, ctypes.POINTER(_I64), ctypes.c_int32, _P, _P, _P]
lib.g5_bfs_batch.restype = ctypes.c_int
lib.g5_bfs_batch_ex.argtypes = [_P, ctypes.POINTER(_I64), ctypes.c_int32, _P, _P, _P,
                                ctypes.POINTER(BatchParams), ctypes.POINTER(BatchStats)]
lib.g5_bfs_batch_ex.restype = ctypes.c_int
lib.g5_bfs_batch_noalloc.argtypes = [_P, ctypes.POINTER(_I64), ctypes.c_int32, _P, _P, _P]
lib.g5_bfs_batch_noalloc.restype = ctypes.c_int
NOALLOC_MAX_N = 1 << 20
lib.g5_build_csr_w.argtypes = [_P, _P, _I64, _I64, _P, _PP]
lib.g5_build_csr_w.restype = ctypes.c_int
lib.g5_csr_copy_weights.argtypes = [_P, _P, _P]
lib.g5_csr_copy_weights.restype = ctypes.c_int


class SsspParams(ctypes.Structure):
    _fields_ = [("delta", ctypes.c_uint32), ("flags", ctypes.c_int32),
                ("pull_div", ctypes.c_int32), ("reserved", ctypes.c_int32 * 5)]


class SsspStats(ctypes.Structure):
    _fields_ = [("rounds", ctypes.c_int64), ("scans", ctypes.c_int64),
                ("buckets", ctypes.c_int64), ("relaxed", ctypes.c_int64),
                ("delta", ctypes.c_int64), ("ms", ctypes.c_double),
                ("edges", ctypes.c_int64), ("pulls", ctypes.c_int64),
                ("reserved", ctypes.c_int64 * 2)]


lib.g5_sssp.argtypes = [_P, _I64, _P, _P, _P]
lib.g5_sssp.restype = ctypes.c_int
lib.g5_sssp_ex.argtypes = [_P, _I64, _P, _P, _P, ctypes.POINTER(SsspParams),
                           ctypes.POINTER(SsspStats)]
lib.g5_sssp_ex.restype = ctypes.c_int
lib.g5_level_work.argtypes = [_P, _P, ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(_I64), _P]
lib.g5_level_work.restype = ctypes.c_int
lib.g5_last_error.argtypes = []
lib.g5_last_error.restype = ctypes.c_char_p


class G5Error(RuntimeError):
    def __init__(self, status, where):
        self.status = status
        msg = (lib.g5_last_error() or b"").decode(errors="replace")
        super().__init__(f"{where}: {STATUS.get(status, status)}: {msg}")


def _check(status, where):
    if status != G5_OK:
        raise G5Error(status, where)


def _stream(device):
    import torch
    return torch.cuda.current_stream(device).cuda_stream


class Csr:
    """A graph built by :func:`build_csr` (device-resident, owned by libg5)."""

    def __init__(self, handle, device):
        self._h = ctypes.c_void_p(handle)
        self.device = device
        n, nnz = _I64(), _I64()
        _check(lib.g5_csr_info(self._h, ctypes.byref(n), ctypes.byref(nnz), None, None),
               "g5_csr_info")
        self.n, self.nnz = n.value, nnz.value

    @property
    def handle(self):
        return self._h

    def arrays(self):
        """Copies of (row_ptr int64[n+1], col_idx int32[nnz]) as device tensors."""
        import torch
        rp = torch.empty(self.n + 1, dtype=torch.int64, device=self.device)
        ci = torch.empty(max(self.nnz, 1), dtype=torch.int32, device=self.device)
        _check(lib.g5_csr_copy(self._h, rp.data_ptr(), ci.data_ptr(), _stream(self.device)),
               "g5_csr_copy")
        return rp, ci[:self.nnz]

    def weights(self):
        """Copy of the edge weights (uint8 [nnz], aligned with col_idx) of a
        graph built by :func:`build_csr_w`, as a device tensor."""
        import torch
        w = torch.empty(max(self.nnz, 1), dtype=torch.uint8, device=self.device)
        _check(lib.g5_csr_copy_weights(self._h, w.data_ptr(), _stream(self.device)),
               "g5_csr_copy_weights")
        return w[:self.nnz]

    def free(self):
        if self._h and self._h.value:
            lib.g5_csr_free(self._h)
            self._h = ctypes.c_void_p(0)

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def build_csr(edges, n):
    """Kernel 1: CSR of a device int64 [m, 2] tuple tensor over n vertices."""
    import torch
    if edges.dtype != torch.int64 or edges.dim() != 2 or edges.shape[1] != 2:
        raise ValueError("edges must be an int64 tensor of shape [m, 2]")
    if not edges.is_cuda:
        raise ValueError("edges must be a device tensor")
    edges = edges.contiguous()
    out = ctypes.c_void_p()
    ptr = edges.data_ptr() if edges.shape[0] else None
    _check(lib.g5_build_csr(ptr, edges.shape[0], int(n), _stream(edges.device),
                            ctypes.byref(out)), "g5_build_csr")
    return Csr(out.value, edges.device)


def build_csr_w(edges, weights, n):
    """Kernel 1 with weights: CSR of a device int64 [m, 2] tuple tensor and a
    device uint8 [m] weight tensor (smallest weight of repeated tuples)."""
    import torch
    if edges.dtype != torch.int64 or edges.dim() != 2 or edges.shape[1] != 2:
        raise ValueError("edges must be an int64 tensor of shape [m, 2]")
    if weights.dtype != torch.uint8 or weights.dim() != 1 or weights.shape[0] != edges.shape[0]:
        raise ValueError("weights must be a uint8 tensor of shape [m]")
    if not edges.is_cuda or not weights.is_cuda:
        raise ValueError("edges and weights must be device tensors")
    edges, weights = edges.contiguous(), weights.contiguous()
    out = ctypes.c_void_p()
    pe = edges.data_ptr() if edges.shape[0] else None
    pw = weights.data_ptr() if edges.shape[0] else None
    _check(lib.g5_build_csr_w(pe, pw, edges.shape[0], int(n), _stream(edges.device),
                              ctypes.byref(out)), "g5_build_csr_w")
    return Csr(out.value, edges.device)


def sssp(csr, src, dist=None, prev=None, delta=None, stats=False, time_call=False,
         pull_div=None):
    """Kernel 3: (dist uint32-as-int32 tensor, prev int32 tensor) from ``src``
    on a graph built by :func:`build_csr_w`.  dist holds uint32 values (0xFFFFFFFF
    = unreached) in an int32 tensor (torch has no uint32 arithmetic); view it
    with ``.cpu().numpy().view(numpy.uint32)``.  ``pull_div``: rounds whose
    queue holds at least nnz / pull_div edges pull (None: the default, a
    negative value: never)."""
    import torch
    if dist is None:
        dist = torch.empty(csr.n, dtype=torch.int32, device=csr.device)
    if prev is None:
        prev = torch.empty(csr.n, dtype=torch.int32, device=csr.device)
    for t in (dist, prev):
        if t.dtype != torch.int32 or t.numel() < csr.n or not t.is_contiguous():
            raise ValueError("dist and prev must be contiguous 32-bit tensors of length n")
    p = SsspParams()
    p.delta = int(delta or 0)
    p.flags = FLAG_TIME_STEPS if time_call else 0
    p.pull_div = int(pull_div or 0)
    st = SsspStats()
    want = stats or time_call
    _check(lib.g5_sssp_ex(csr.handle, int(src), dist.data_ptr(), prev.data_ptr(),
                          _stream(csr.device), ctypes.byref(p), ctypes.byref(st) if want else None),
           "g5_sssp")
    if not want:
        return dist, prev
    info = {k: getattr(st, k) for k in ("rounds", "scans", "buckets", "relaxed", "edges", "delta",
                                        "ms", "pulls")}
    return dist, prev, info


def _params(direction, alpha, beta, lane_scan, claim, flags, blocks_per_cu=None, lds_kb=None,
            lds_density=None, vertices_per_lane=None, td_blocks_per_cu=None, gamma=None,
            heavy_kedges=None):
    p = BfsParams()
    p.heavy_kedges = heavy_kedges or 0
    p.bu_vertices_per_lane = vertices_per_lane or 0
    p.td_blocks_per_cu = td_blocks_per_cu or 0
    p.gamma = gamma or 0.0
    p.direction = direction
    p.alpha = alpha or 0.0
    p.beta = beta or 0.0
    p.lds_density = lds_density or 0.0
    p.bu_lane_scan = lane_scan or 0
    p.claim = claim
    p.flags = flags
    p.bu_blocks_per_cu = blocks_per_cu or 0
    p.lds_kb = lds_kb or 0
    return p


def bfs(csr, root, parent=None, level=None, direction=DIR_AUTO, alpha=None, beta=None,
        lane_scan=None, claim=CLAIM_OR, hint=True, packed=None, min_parent=False, lds=True,
        blocks_per_cu=None, lds_kb=None, lds_density=None, vertices_per_lane=None,
        td_blocks_per_cu=None, gamma=None, heavy_kedges=None, stats=False,
        time_steps=False, count_bytes=False):
    """Kernel 2: (parent, level) int32 device tensors of length n from ``root``.

    With ``stats=True`` also returns a dict of per-level directions, frontier
    sizes and discoveries; ``time_steps`` adds each step kernel's device time
    (HIP events carried by its dispatch on the current stream) and ``count_bytes`` its algorithmic bytes.
    """
    import torch
    if parent is None:
        parent = torch.empty(csr.n, dtype=torch.int32, device=csr.device)
    if level is None:
        level = torch.empty(csr.n, dtype=torch.int32, device=csr.device)
    for t in (parent, level):
        if t.dtype != torch.int32 or t.numel() < csr.n or not t.is_contiguous():
            raise ValueError("parent and level must be contiguous int32 tensors of length n")
    flags = ((FLAG_TIME_STEPS if time_steps else 0) | (FLAG_COUNT_BYTES if count_bytes else 0)
             | (0 if hint else FLAG_NO_HINT)
             | {None: 0, True: FLAG_PACKED, False: FLAG_ROWLOOP}[packed]
             | (FLAG_MIN_PARENT if min_parent else 0) | (0 if lds else FLAG_NO_LDS))
    p = _params(direction, alpha, beta, lane_scan, claim, flags, blocks_per_cu, lds_kb,
                lds_density, vertices_per_lane, td_blocks_per_cu, gamma, heavy_kedges)
    want = stats or time_steps or count_bytes
    st = BfsStats()
    _check(lib.g5_bfs_ex(csr.handle, int(root), parent.data_ptr(), level.data_ptr(),
                         _stream(csr.device), ctypes.byref(p),
                         ctypes.byref(st) if want else None), "g5_bfs")
    if not want:
        return parent, level
    nl = min(st.nlevels, MAX_STAT_LEVELS)
    info = {"nlevels": st.nlevels, "reached": st.reached, "alpha": st.alpha, "beta": st.beta,
            "lane_scan": st.bu_lane_scan, "blocks_per_cu": st.bu_blocks_per_cu,
            "lds_levels": st.lds_levels, "lds_shift": st.lds_shift,
            "lds_mask": st.lds_mask & ((1 << 64) - 1),
            "heavy_mask": st.heavy_mask & ((1 << 64) - 1)}
    for k in ("dir", "frontier", "discovered", "edges", "bytes", "step_ms"):
        info[k] = list(getattr(st, k)[:nl])
    return parent, level, info


def bfs_batch(csr, roots, parents=True, levels=None, parent_out=None, direction=DIR_AUTO,
              alpha=None, blocks_per_cu=None, stepped=True, persistent=False, stats=False,
              time_launch=False, graph=False):
    """Batched BFS from 1..64 roots, one plain launch per level (these may
    overlap other streams' work); ``persistent=True``: every level in one
    cooperative launch; ``graph=True``: the level loop as replays of one HIP
    graph of 8 level kernels.  ``stepped`` is accepted for older callers.

    Returns (parents int32 [k, n] or None, levels int8 [k, n]) and, with
    ``stats=True``, a dict of per-level directions and frontier sizes.
    """
    import torch
    k = len(roots)
    arr = (_I64 * max(k, 1))(*[int(r) for r in roots])
    if levels is None:
        levels = torch.empty((k, csr.n), dtype=torch.int8, device=csr.device)
    if parents and parent_out is None:
        parent_out = torch.empty((k, csr.n), dtype=torch.int32, device=csr.device)
    for t, dt in ((levels, torch.int8), (parent_out if parents else None, torch.int32)):
        if t is not None and (t.dtype != dt or t.numel() < k * csr.n or not t.is_contiguous()):
            raise ValueError("levels must be contiguous int8 [k, n] and parents int32 [k, n]")
    pp = parent_out.data_ptr() if parents else None
    p = BatchParams()
    p.direction = direction
    p.alpha = alpha or 0.0
    p.flags = ((FLAG_TIME_STEPS if time_launch else 0) | (FLAG_STEPPED if stepped else 0)
               | (FLAG_PERSISTENT if persistent else 0) | (FLAG_GRAPH if graph else 0))
    p.blocks_per_cu = blocks_per_cu or 0
    st = BatchStats()
    want = stats or time_launch
    _check(lib.g5_bfs_batch_ex(csr.handle, arr, k, pp, levels.data_ptr(), _stream(csr.device),
                               ctypes.byref(p), ctypes.byref(st) if want else None),
           "g5_bfs_batch")
    out = (parent_out if parents else None), levels
    if not want:
        return out
    nl = min(st.nlevels, MAX_STAT_LEVELS)
    info = {"nlevels": st.nlevels, "dir": list(st.dir[:nl]), "frontier": list(st.frontier[:nl]),
            "launch_ms": st.launch_ms, "grid_blocks": st.grid_blocks, "alpha": st.alpha}
    return out + (info,)


def level_work(csr, level, lvl, bottom_up=True):
    """Work counts of level ``lvl`` of a finished traversal (measurement):
    dict with q, mf, claimed, unvisited, scanned (see g5_level_work); the last
    two only with ``bottom_up``."""
    import torch
    if level.dtype != torch.int32 or level.numel() < csr.n or not level.is_contiguous():
        raise ValueError("level must be a contiguous int32 tensor of length n")
    out = (_I64 * 5)()
    _check(lib.g5_level_work(csr.handle, level.data_ptr(), int(lvl), int(bool(bottom_up)), out,
                             _stream(csr.device)), "g5_level_work")
    return dict(zip(("q", "mf", "claimed", "unvisited", "scanned"), list(out)))


def bfs_batch_noalloc(csr, roots, parents=True, levels=None, parent_out=None):
    """g5_bfs_batch_noalloc: the batched traversal on the library's fixed
    workspace (graphs of at most NOALLOC_MAX_N vertices); the output tensors
    are the caller's.  Returns (parents or None, levels)."""
    import torch
    k = len(roots)
    arr = (_I64 * max(k, 1))(*[int(r) for r in roots])
    if levels is None:
        levels = torch.empty((k, csr.n), dtype=torch.int8, device=csr.device)
    if parents and parent_out is None:
        parent_out = torch.empty((k, csr.n), dtype=torch.int32, device=csr.device)
    for t, dt in ((levels, torch.int8), (parent_out if parents else None, torch.int32)):
        if t is not None and (t.dtype != dt or t.numel() < k * csr.n or not t.is_contiguous()):
            raise ValueError("levels must be contiguous int8 [k, n] and parents int32 [k, n]")
    pp = parent_out.data_ptr() if parents else None
    _check(lib.g5_bfs_batch_noalloc(csr.handle, arr, k, pp, levels.data_ptr(),
                                    _stream(csr.device)), "g5_bfs_batch_noalloc")
    return (parent_out if parents else None), levels
