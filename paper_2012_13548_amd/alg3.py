"""Host experiment: the paper's level-synchronous parallel BFS (Algorithm 3,
Section 2.3.2) with OpenMP threads, through libg5alg3.so (include/g5_alg3.h),
for a speedup curve over thread counts.  Separate from the GPU path: the GPU
entry points never call it."""
import ctypes
import os

import numpy as np

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libg5alg3.so")
_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise RuntimeError(f"{_LIB_PATH} is not built (run __graft_entry__.build())")
        _lib = ctypes.CDLL(_LIB_PATH)
        _lib.g5_alg3_bfs.restype = ctypes.c_int
        _lib.g5_alg3_bfs.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                     ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                                     ctypes.c_int, ctypes.POINTER(ctypes.c_double)]
    return _lib


def bfs(row_ptr, col_idx, root, threads):
    """(parent, level, seconds) from `root` with `threads` OpenMP threads;
    row_ptr int64 [n + 1], col_idx int32 [nnz] (numpy, host)."""
    rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
    ci = np.ascontiguousarray(col_idx, dtype=np.int32)
    n = rp.size - 1
    level = np.empty(n, dtype=np.int32)
    parent = np.empty(n, dtype=np.int32)
    sec = ctypes.c_double(0.0)
    st = _load().g5_alg3_bfs(rp.ctypes.data, ci.ctypes.data, n, int(root), level.ctypes.data,
                             parent.ctypes.data, int(threads), ctypes.byref(sec))
    if st != 0:
        raise ValueError(f"g5_alg3_bfs failed with status {st}")
    return parent, level, sec.value
