"""The C-ABI library loads and exports every symbol include/g5.h declares
(no GPU needed: nothing is called that touches the device)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "g5.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(g5_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    syms = declared_symbols()
    for s in ["g5_build_csr", "g5_csr_info", "g5_csr_copy", "g5_csr_free", "g5_bfs",
              "g5_bfs_ex", "g5_bfs_batch", "g5_last_error", "g5_build_csr_w", "g5_sssp",
              "g5_sssp_ex", "g5_csr_copy_weights", "g5_level_work"]:
        assert s in syms


def test_library_exports_every_declared_symbol():
    import paper_2012_13548_amd as g5
    lib = ctypes.CDLL(g5.LIB_PATH)
    for s in declared_symbols():
        assert hasattr(lib, s), s


def test_null_arguments_rejected_without_device():
    import paper_2012_13548_amd as g5
    lib = g5.lib
    assert lib.g5_bfs(None, 0, None, None, None) == g5.G5_EINVAL
    assert b"non-NULL" in lib.g5_last_error()
    assert lib.g5_csr_info(None, None, None, None, None) == g5.G5_EINVAL
    assert lib.g5_bfs_batch(None, None, 1, None, None, None) == g5.G5_EINVAL
    assert lib.g5_build_csr(None, 0, 4, None, None) == g5.G5_EINVAL
    assert lib.g5_sssp(None, 0, None, None, None) == g5.G5_EINVAL
    assert lib.g5_build_csr_w(None, None, 0, 4, None, None) == g5.G5_EINVAL
    assert lib.g5_level_work(None, None, 0, 1, None, None) == g5.G5_EINVAL
    lib.g5_csr_free(None)


def test_generator_device_library_loads():
    import kronecker as K
    lib = K._load_dev()
    assert hasattr(lib, "kron_edges_device") and hasattr(lib, "kron_nonisolated_device")


def test_struct_layouts_match_header(tmp_path):
    # the ctypes mirrors of the parameter and statistics structs have the C sizes
    import subprocess
    import paper_2012_13548_amd as g5
    src = tmp_path / "sizes.c"
    src.write_text('#include <stdio.h>\n#include "g5.h"\nint main(void){printf("%zu %zu %zu %zu %zu %zu",'
                   ' sizeof(g5_bfs_params), sizeof(g5_bfs_stats), sizeof(g5_batch_params),'
                   ' sizeof(g5_batch_stats), sizeof(g5_sssp_params), sizeof(g5_sssp_stats));'
                   'return 0;}\n')
    exe = tmp_path / "sizes"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(src)],
                   check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()
    assert [int(x) for x in out] == [ctypes.sizeof(g5.BfsParams), ctypes.sizeof(g5.BfsStats),
                                     ctypes.sizeof(g5.BatchParams), ctypes.sizeof(g5.BatchStats),
                                     ctypes.sizeof(g5.SsspParams), ctypes.sizeof(g5.SsspStats)]
