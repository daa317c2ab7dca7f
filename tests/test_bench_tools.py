"""Host logic of the benchmark's measurement tools, on synthetic inputs: the
rocprofv3 counter reduction (calibration by the copy probe, the dispatches it
keeps and drops, traversal counting, the per-level split of the last
traversal), the source-hash gate on the stored
record, and the kernel-trace summary."""
import csv
import json
import os
import sqlite3

import bench

KIB = 1024
HEAD = ["Correlation_Id", "Dispatch_Id", "Agent_Id", "Queue_Id", "Process_Id", "Thread_Id",
        "Grid_Size", "Kernel_Id", "Kernel_Name", "Workgroup_Size", "LDS_Block_Size",
        "Scratch_Size", "VGPR_Count", "Accum_VGPR_Count", "SGPR_Count", "Counter_Name",
        "Counter_Value", "Start_Timestamp", "End_Timestamp"]
COPY = "void at::native::vectorized_elementwise_kernel<4, at::native::CUDAFunctorOnSelf_add<long>>"
BU = "void g5::(anonymous namespace)::k_bu_step<8, 1, false>(unsigned int const*)"
BU_ACCT = "void g5::(anonymous namespace)::k_bu_step<8, 1, true>(unsigned int const*)"
BU_LDS = "void g5::(anonymous namespace)::k_bu_step_lds<4, 1, false>(unsigned int const*)"
TD = "void g5::(anonymous namespace)::k_td_expand<0>(int const*)"
INIT = "g5::(anonymous namespace)::k_bfs_init(long, unsigned char*)"


def write_run(d, counter, dispatches):
    """dispatches: (id, kernel, grid, [values in KiB, one row each])."""
    os.makedirs(os.path.join(d, "host"), exist_ok=True)
    with open(os.path.join(d, "host", "run_counter_collection.csv"), "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(HEAD)
        for i, name, grid, vals in dispatches:
            for v in vals:
                w.writerow([i, i, "Agent 1", 1, 1, 1, grid, 7, name, 256, 0, 0, 32, 0, 96,
                            counter, v, 0, 1])


def test_reduce_pmc(tmp_path):
    n = 1 << 10
    copy_f = bench.COPY_PROBE_BYTES / 2 / KIB  # FETCH_SIZE reads half of the bytes
    copy_w = bench.COPY_PROBE_BYTES / KIB
    fetch = [(1, COPY, 8, [copy_f / 2, copy_f / 2]),  # one value per XCD, summed
             (2, INIT, 1 << 20, [10]), (3, INIT, 1 << 20, [10]), (4, INIT, 256, [1]),
             (5, BU, 99, [2000]), (6, BU, 99, [4000]), (7, BU, 99, [10]),  # 7: queued ahead
             (8, BU_ACCT, 99, [9e6]),
             (9, TD, 99, [100]), (10, TD, 99, [300]), (11, TD, 99, [1])]
    write = [(1, COPY, 8, [copy_w]),
             (2, INIT, 1 << 20, [10]), (3, INIT, 1 << 20, [10]), (4, INIT, 256, [1]),
             (5, BU, 99, [1500]), (6, BU, 99, [2500]), (7, BU, 99, [0]), (8, BU_ACCT, 99, [9e6]),
             (9, TD, 99, [50]), (10, TD, 99, [70]), (11, TD, 99, [4])]  # 11 finishes a traversal
    fetch += [(12, BU_LDS, 99, [8000])]
    write += [(12, BU_LDS, 99, [3000])]
    split = [(1, COPY, 8, [100]), (5, BU, 99, [40]), (6, BU, 99, [60]), (7, BU, 99, [1]),
             (12, BU_LDS, 99, [70])]
    write_run(str(tmp_path / "f"), "FETCH_SIZE", fetch)
    write_run(str(tmp_path / "w"), "WRITE_SIZE", write)
    for c in bench.SPLIT_COUNTERS:
        write_run(str(tmp_path / "s" / c), c, split)
    # the three split counters in one run directory
    rows = []
    for c in bench.SPLIT_COUNTERS:
        rows += list(csv.reader(open(str(tmp_path / "s" / c / "host" /
                                         "run_counter_collection.csv"))))[1:]
    os.makedirs(str(tmp_path / "sp" / "host"))
    with open(str(tmp_path / "sp" / "host" / "run_counter_collection.csv"), "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(HEAD)
        w.writerows(rows)
    out = str(tmp_path / "traffic.json")
    bench.reduce_pmc(str(tmp_path / "f"), str(tmp_path / "w"), str(tmp_path / "sp"), "s10", "cmd",
                     path=out)
    data = json.load(open(out))
    bu, td, lds = data["k_bu_step@s10"], data["k_td_expand@s10"], data["k_bu_step_lds@s10"]
    assert bu["fetch_factor"] == 2.0 and bu["write_factor"] == 1.0
    # working bottom-up dispatches only: (2000 + 4000) / 2 KiB fetched, x2; (1500 + 2500) / 2 written
    assert bu["fetch_bytes_per_launch"] == 6000 * KIB
    assert bu["write_bytes_per_launch"] == 2000 * KIB
    assert bu["bytes_per_launch"] == 8000 * KIB and bu["launches"] == [2, 2]
    assert bu["raw_bytes_per_launch"] == (3000 + 2000) * KIB
    assert bu["read_requests_per_launch"]["TCC_EA0_RDREQ_sum"] == 50  # (40 + 60) / 2
    assert bu["read_requests_per_launch"]["copy_probe"]["TCC_EA0_RDREQ_sum"] == 100
    assert lds["bytes_per_launch"] == (2 * 8000 + 3000) * KIB and lds["launches"] == [1, 1]
    # two traversals of the workload graph (the small-grid init is a warm-up); the
    # finishing dispatch (writes >= 4n bytes, fetches less) is left out
    assert td["traversals"] == 2 and td["finishing_dispatches"] == 1 and td["dispatches"] == 3
    assert td["fetch_bytes_per_traversal"] == (100 + 300) * 2 * KIB // 2
    assert td["write_bytes_per_traversal"] == (50 + 70) * KIB // 2
    assert td["source_hash"] == bench.source_hash(bench.BFS_SOURCES)
    assert bench.measured_traffic("k_bu_step", "s10", path=out) == 8000 * KIB
    assert bench.measured_traffic("k_td_expand", "s10", "bytes_per_traversal", path=out) == \
        td["bytes_per_traversal"]
    assert bench.measured_traffic("k_bu_step", "s26", path=out) is None
    # the last workload traversal's levels: working step dispatches in order, without
    # the queued-ahead step (writes nothing), the byte-counting variant and the finish
    levels = bench.measured_traffic("root0_levels", "s10", "levels", path=out)
    assert [x["dir"] for x in levels] == ["BU", "BU", "TD", "TD", "BU"]
    assert [x["bytes"] for x in levels] == [(2 * 2000 + 1500) * KIB, (2 * 4000 + 2500) * KIB,
                                            (2 * 100 + 50) * KIB, (2 * 300 + 70) * KIB,
                                            (2 * 8000 + 3000) * KIB]


def test_traffic_gated_by_source_hash(tmp_path):
    out = str(tmp_path / "traffic.json")
    rec = {"source_hash": "not-this-source", "bytes_per_launch": 5}
    json.dump({"k_bu_step@s26": rec}, open(out, "w"))
    assert bench.measured_traffic("k_bu_step", "s26", path=out) is None
    rec["source_hash"] = bench.source_hash(bench.BFS_SOURCES)
    json.dump({"k_bu_step@s26": rec}, open(out, "w"))
    assert bench.measured_traffic("k_bu_step", "s26", path=out) == 5
    assert bench.measured_traffic("k_bu_step", "s26", path=str(tmp_path / "none.json")) is None


def test_summarize_trace(tmp_path, capsys):
    db = str(tmp_path / "run_results.db")
    c = sqlite3.connect(db)
    c.execute("create table kernels (name text, start integer, end integer)")
    us = 1000  # the trace's timestamps are in ns
    rows = [(BU, 0, 200 * us), (BU, 0, 100 * us), (BU, 0, 3 * us),  # the last exited at once
            (BU_LDS, 0, 300 * us), (BU_ACCT, 0, 900 * us), (TD, 0, 50 * us)]
    c.executemany("insert into kernels values (?, ?, ?)", rows)
    c.commit()
    c.close()
    line = {"roofline": {"kernel": "k_bu_step", "launches": 3, "avg_launch_ms": 0.2},
            "step_kernels": {"k_bu_step_lds": {"all": {"launches": 1, "ms": 0.3}}}}
    bj = str(tmp_path / "bench.json")
    open(bj, "w").write("progress\n" + json.dumps(line) + "\n")
    bench.summarize_trace(db, "the command", bj)
    md = capsys.readouterr().out
    assert "the command" in md
    assert "* dispatches: 3, of which 1 are steps queued ahead" in md
    assert "* working dispatches: 2, average 150.00 us" in md
    assert "* working dispatches: 1, average 300.00 us" in md
    assert "avg_launch_ms 0.2" in md
    assert "| `k_bu_step<8, 1, false>` | 3 | 303.0 | 101.00 |" in md
    assert "## k_bu_step_lds" in md and "1 instrumented launches, 0.3 ms" in md
