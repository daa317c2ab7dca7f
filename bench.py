#!/usr/bin/env python3
"""Benchmark: harmonic-mean GTEPS of single-root BFS on a scale-26, edge-factor-16
Kronecker graph over 64 roots, on one MI355X.

One step = one breadth-first search from each of the 64 roots (g5_bfs through
the C-ABI).  Inputs are generated straight into HBM (seeded Kronecker
generator, initiator 0.57/0.19/0.19/0.05, random relabel) and the CSR is built
by g5_build_csr before timing; the CSR build is timed separately.

Per root r: t_r = device time of g5_bfs (events on the launch stream around
the call), m_r = distinct undirected edges of r's component, TEPS_r = m_r/t_r.
value = harmonic mean of TEPS over every (step, root) sample (Section 4.3 of
the paper names TEPS over 64 start vertices as the Graph500 metric).

Printed JSON line (stdout): the contract fields plus
  roofline      the dominant step kernel's algorithmic GB/s vs the 8 TB/s peak
                (kernel durations from an instrumented pass after the timed steps)
  cpu_baseline  the CPU oracle (single-threaded queue BFS) timed on this host
                on a bounded sample (some roots of the same graph)
  batch         64 roots in one batched launch vs 64 sequential runs (scale 22)
Progress goes to stderr.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "harmonic-mean GTEPS, scale-26 ef16, 64 roots; batched vs single-root; HBM GB/s"
T0 = time.time()


def log(msg):
    sys.stderr.write(f"[bench {time.time() - T0:7.1f}s] {msg}\n")
    sys.stderr.flush()


def hmean(xs):
    return len(xs) / sum(1.0 / x for x in xs)


def source_hash(paths):
    h = hashlib.sha256()
    for p in paths:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


BFS_SOURCES = ["paper_2012_13548_amd/csrc/bfs.hip", "paper_2012_13548_amd/csrc/g5_internal.h",
               "paper_2012_13548_amd/csrc/tuned_table.inc"]


TRAFFIC_PATH = os.path.join(ROOT, "profiles", "traffic.json")


def measured_traffic(kernel, workload, field="bytes_per_launch", path=TRAFFIC_PATH):
    """HBM bytes (per launch, or the record's `field`) from committed rocprofv3
    counter runs, if they were taken on the current kernel source (else None)."""
    if not os.path.exists(path):
        return None
    with open(path) as f:
        data = json.load(f)
    rec = data.get(f"{kernel}@{workload}")
    if not rec or rec.get("source_hash") != source_hash(BFS_SOURCES):
        return None
    return rec.get(field)


COPY_PROBE_BYTES = 1 << 31  # each direction


def copy_probe():
    """A plain elementwise copy of known size (2 GiB read, 2 GiB written): the
    calibration dispatch for the rocprofv3 FETCH_SIZE / WRITE_SIZE counters."""
    import torch
    src = torch.ones(COPY_PROBE_BYTES // 8, dtype=torch.int64, device="cuda:0")
    dst = torch.empty_like(src)
    torch.add(src, 0, out=dst)
    torch.cuda.synchronize()
    del src, dst
    torch.cuda.empty_cache()


GATHER_ELEMS = 1 << 29   # int64 source: 4 GiB
GATHER_PICKS = 1 << 24   # random reads


def gather_probe():
    """A random gather of known footprint: 2^24 int64 elements picked at
    seeded random positions of a 4 GiB array (torch.take), for calibrating the
    read counters on small random requests.  Prints the distinct 64-byte lines
    it touches and the bytes of its index and output streams."""
    import torch
    src = torch.zeros(GATHER_ELEMS, dtype=torch.int64, device="cuda:0")
    gen = torch.Generator(device="cuda:0")
    gen.manual_seed(5)
    idx = torch.randint(0, GATHER_ELEMS, (GATHER_PICKS,), generator=gen, device="cuda:0")
    torch.cuda.synchronize()
    out = torch.take(src, idx)
    torch.cuda.synchronize()
    lines = int(torch.unique(idx // 8).numel())
    log(json.dumps({"gather_probe": {"distinct_lines": lines, "line_bytes": 64,
                                     "index_bytes": GATHER_PICKS * 8,
                                     "out_bytes": GATHER_PICKS * 8}}))
    del src, idx, out
    torch.cuda.empty_cache()


def _pmc_rows(d):
    import csv
    import glob
    files = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise SystemExit(f"no counter_collection.csv under {d}")
    with open(files[0]) as f:
        return list(csv.DictReader(f))


def _per_dispatch(rows, counter, match, largest=False, min_kib=0.0):
    """Average (or, with largest, maximum) of `counter` (KiB) over dispatches
    whose kernel name satisfies match and whose value exceeds min_kib."""
    per = {}
    for r in rows:
        if r.get("Counter_Name") != counter or not match(r.get("Kernel_Name", "")):
            continue
        key = r.get("Dispatch_Id") or r.get("Correlation_Id")
        per[key] = per.get(key, 0.0) + float(r["Counter_Value"])
    per = {k: v for k, v in per.items() if v > min_kib}
    if not per:
        raise SystemExit(f"no {counter} samples for the requested kernel")
    if largest:
        return max(per.values()), 1
    return sum(per.values()) / len(per), len(per)


def _per_dispatch_map(rows, counter, match):
    """{dispatch id: counter value in KiB} over dispatches of matching kernels."""
    per = {}
    for r in rows:
        if r.get("Counter_Name") != counter or not match(r.get("Kernel_Name", "")):
            continue
        key = int(r.get("Dispatch_Id") or r.get("Correlation_Id"))
        per[key] = per.get(key, 0.0) + float(r["Counter_Value"])
    return per


def step_kernel_of(name):
    """The step kernel a dispatch belongs to (k_bu_step, k_bu_step_lds or
    k_td_expand), or None; the byte-counting variants of the bottom-up steps
    (third template argument true) belong to none."""
    import re
    m = re.search(r"k_bu_step(_lds)?<\d+, \d+, (true|false)", name)
    if m:
        return None if m.group(2) == "true" else ("k_bu_step_lds" if m.group(1) else "k_bu_step")
    return "k_td_expand" if "k_td_expand<" in name else None


def is_bu_step(name):
    return step_kernel_of(name) in ("k_bu_step", "k_bu_step_lds")


# A bottom-up step queued ahead of the host's decision exits at once when the
# level turns top-down; such dispatches move no data (a working one at least
# reads and writes the visited and next-frontier words).
NOOP_KIB = 1024.0
NOOP_US = 10.0
# request-size split of the reads that leave L2 (FETCH_SIZE is derived from
# these: 128 B per TCC_BUBBLE, 32 B per TCC_EA0_RDREQ_32B, 64 B for the rest)
SPLIT_COUNTERS = ("TCC_EA0_RDREQ_sum", "TCC_EA0_RDREQ_32B_sum", "TCC_BUBBLE_sum")


def reduce_pmc(fetch_dir, write_dir, split_dir, workload, command, path=TRAFFIC_PATH):
    """HBM bytes per working launch of each bottom-up step kernel (and per
    traversal of the top-down expansions) from a FETCH_SIZE run, a WRITE_SIZE
    run and a run of the read-request counters split by size.  Each of
    FETCH_SIZE and WRITE_SIZE is scaled by what it reads for the copy probe
    (known bytes); the raw counter values and the request split are kept
    beside.  Stored in profiles/traffic.json with the kernel source hash, so
    the bench reports them only while the kernels are unchanged."""
    # the copy probe: torch's elementwise add over 2 GiB, the largest such dispatch
    is_copy = lambda name: "elementwise_kernel" in name and "_add<long>" in name
    fr, wr = _pmc_rows(fetch_dir), _pmc_rows(write_dir)
    sr = _pmc_rows(split_dir) if split_dir else []
    copy_f, _ = _per_dispatch(fr, "FETCH_SIZE", is_copy, largest=True)
    copy_w, _ = _per_dispatch(wr, "WRITE_SIZE", is_copy, largest=True)
    f_factor = COPY_PROBE_BYTES / (copy_f * 1024)
    w_factor = COPY_PROBE_BYTES / (copy_w * 1024)
    h = source_hash(BFS_SOURCES)
    data = {}
    if os.path.exists(path):
        with open(path) as f:
            data = json.load(f)

    def split_of(match, keys=None):
        out = {}
        for c in SPLIT_COUNTERS:
            per = _per_dispatch_map(sr, c, match)
            if keys is not None:
                per = {k: v for k, v in per.items() if k in keys}
            out[c] = int(sum(per.values()) / max(len(per), 1)) if per else None
        if sr and copy_split:
            out["copy_probe"] = copy_split
        return out

    copy_split = {}
    if sr:
        for c in SPLIT_COUNTERS:
            per = _per_dispatch_map(sr, c, is_copy)
            copy_split[c] = int(max(per.values())) if per else None
    recs = []
    for kernel in ("k_bu_step", "k_bu_step_lds"):
        match = (lambda k: (lambda name: step_kernel_of(name) == k))(kernel)
        fm = {k: v for k, v in _per_dispatch_map(fr, "FETCH_SIZE", match).items() if v > NOOP_KIB}
        wm = _per_dispatch_map(wr, "WRITE_SIZE", match)
        wm = {k: v for k, v in wm.items() if k in fm}
        if not fm:
            continue
        kf = sum(fm.values()) / len(fm)
        kw = sum(wm.values()) / max(len(wm), 1)
        rec = {"source_hash": h,
               "bytes_per_launch": int(kf * 1024 * f_factor + kw * 1024 * w_factor),
               "fetch_bytes_per_launch": int(kf * 1024 * f_factor),
               "write_bytes_per_launch": int(kw * 1024 * w_factor),
               "raw_bytes_per_launch": int((kf + kw) * 1024),
               "fetch_factor": round(f_factor, 4), "write_factor": round(w_factor, 4),
               "launches": [len(fm), len(wm)],
               "read_requests_per_launch": split_of(match, set(fm)) if sr else None,
               "command": command}
        data[f"{kernel}@{workload}"] = rec
        recs.append((kernel, rec))

    # The top-down expansion: its launches include those queued ahead that did
    # nothing and, once per traversal, the one that finishes it (widens the
    # byte levels into the int32 level array: it writes ~4n bytes and fetches
    # less than it writes), which belongs to no top-down level.  Both runs
    # execute the same program, so dispatch ids match between them; the
    # record is the traffic of the real expansions per traversal (the bench
    # divides it by its own count of top-down levels per traversal).
    is_td = lambda name: step_kernel_of(name) == "k_td_expand"
    tf = _per_dispatch_map(fr, "FETCH_SIZE", is_td)
    tw = _per_dispatch_map(wr, "WRITE_SIZE", is_td)
    if set(tf) != set(tw):
        raise SystemExit("the two counter runs dispatched different top-down expansions")
    # traversals of the workload graph: init dispatches of the largest grid (the
    # run also warms the kernels up on a small graph)
    grids = {int(r["Dispatch_Id"]): int(r["Grid_Size"]) for r in fr
             if r.get("Counter_Name") == "FETCH_SIZE" and "k_bfs_init" in r.get("Kernel_Name", "")}
    inits = sum(1 for g in grids.values() if g == max(grids.values()))
    n = 1 << int(workload.lstrip("s"))
    ending = {k for k in tw
              if tw[k] * 1024 * w_factor >= 0.9 * 4 * n and tf[k] * f_factor < tw[k] * w_factor}
    td_f = sum(v for k, v in tf.items() if k not in ending) * 1024 * f_factor
    td_w = sum(v for k, v in tw.items() if k not in ending) * 1024 * w_factor
    td_raw = (sum(v for k, v in tf.items() if k not in ending)
              + sum(v for k, v in tw.items() if k not in ending)) * 1024
    td = {"source_hash": h,
          "bytes_per_traversal": int((td_f + td_w) / inits),
          "fetch_bytes_per_traversal": int(td_f / inits),
          "write_bytes_per_traversal": int(td_w / inits),
          "raw_bytes_per_traversal": int(td_raw / inits),
          "traversals": inits, "dispatches": len(tf), "finishing_dispatches": len(ending),
          "command": command}
    data[f"k_td_expand@{workload}"] = td

    # Per level: the run's last traversal of the workload graph is a plain one
    # from the benchmark's first root.  Its step kernels in dispatch order are
    # its levels, leaving out the steps queued ahead that exited at once (they
    # write nothing) and the dispatch that finishes the traversal.
    last = max(k for k, g in grids.items() if g == max(grids.values()))
    names = {int(r["Dispatch_Id"]): r.get("Kernel_Name", "") for r in fr}
    fa = _per_dispatch_map(fr, "FETCH_SIZE", lambda name: True)
    wa = _per_dispatch_map(wr, "WRITE_SIZE", lambda name: True)
    levels = []
    for k in sorted(d for d in fa if d > last):
        name = names[k]
        if not (is_td(name) or is_bu_step(name)) or wa.get(k, 0.0) <= 0 or k in ending:
            continue
        levels.append({"dir": "TD" if is_td(name) else "BU",
                       "bytes": int(fa[k] * 1024 * f_factor + wa[k] * 1024 * w_factor),
                       "raw_bytes": int((fa[k] + wa[k]) * 1024)})
    data[f"root0_levels@{workload}"] = {"source_hash": h, "levels": levels, "command": command}
    data.pop("k_bu_step_all@" + workload, None)
    data.pop("td_step@" + workload, None)
    if sr:
        g = gather_calibration(fr, sr, copy_split)
        if g:
            data["gather_probe"] = dict(g, command=command)
    with open(path, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    for kernel, rec in recs:
        print(kernel, json.dumps(rec))
    print(json.dumps(td))
    print(json.dumps(levels))


def gather_calibration(fr, sr, copy_split):
    """Read requests of the random-gather probe (when the counter runs include
    it): the copy probe gives the bytes one request moves on a stream; the
    gather's requests beyond those of its index stream, per random pick, show
    whether scattered 8-byte reads cost one such request each."""
    # the probe's gather is the run's first indexing dispatch (the probes run
    # before the workload)
    is_take = lambda name: "index_elementwise_kernel" in name
    req = _per_dispatch_map(sr, "TCC_EA0_RDREQ_sum", is_take)
    fetch = _per_dispatch_map(fr, "FETCH_SIZE", is_take)
    copy_req = copy_split.get("TCC_EA0_RDREQ_sum")
    if not req or not copy_req:
        return None
    r = req[min(req)]
    per_req = COPY_PROBE_BYTES / copy_req
    index_req = GATHER_PICKS * 8 / per_req
    return {"picks": GATHER_PICKS, "read_requests": int(r),
            "stream_bytes_per_request": round(per_req, 2),
            "index_requests": int(index_req),
            "requests_per_pick": round((r - index_req) / GATHER_PICKS, 4),
            "fetch_size_kib": round(fetch[min(fetch)], 1) if fetch else None}


def summarize_trace(db, command, bench_json=None,
                    title="Kernel trace: scale-26 single-root BFS benchmark"):
    """Markdown summary of a rocprofv3 kernel trace (its SQLite database): the
    busiest kernels, and each step kernel's average over working launches,
    which is what the bench's avg_launch_ms measures with HIP events."""
    import re
    import sqlite3
    c = sqlite3.connect(db)
    rows = list(c.execute("select name, start, end from kernels"))

    def short(n):
        n = n.replace("g5::(anonymous namespace)::", "").replace("void ", "")
        return re.sub(r"\(.*$", "", n)[:60]

    agg = {}
    for name, t0, t1 in rows:
        a = agg.setdefault(short(name), [0, 0.0])
        a[0] += 1
        a[1] += (t1 - t0) / 1e3
    total = sum(a[1] for a in agg.values())
    out = [f"# {title}", "",
           "Command (from the repository root):", "", "```", command, "```", "",
           "Durations are rocprofv3 kernel-trace dispatch times (microseconds), over the",
           "whole command (graph generation and CSR build, accounting pass, warm-up and",
           "timed steps, and any batch run or probe it includes).", "",
           "| kernel | calls | total us | avg us | % |", "|---|---:|---:|---:|---:|"]
    for k, (n, t) in sorted(agg.items(), key=lambda kv: -kv[1][1])[:24]:
        out.append(f"| `{k}` | {n} | {t:.1f} | {t / n:.2f} | {100 * t / total:.1f} |")
    bench = None
    if bench_json:
        with open(bench_json) as f:
            line = [l for l in f if l.startswith("{")][-1]
        bench = json.loads(line)
    for kernel in ("k_bu_step", "k_bu_step_lds"):
        d = [(t1 - t0) / 1e3 for name, t0, t1 in rows if step_kernel_of(name) == kernel]
        if not d:
            continue
        work = [x for x in d if x > NOOP_US]
        out += ["", f"## {kernel} (timed variant, without byte counting)", "",
                f"* dispatches: {len(d)}, of which {len(d) - len(work)} are steps queued ahead "
                f"that exited at once (< {NOOP_US:.0f} us)",
                f"* working dispatches: {len(work)}, average {sum(work) / max(len(work), 1):.2f} us"]
        if bench:
            r = bench["roofline"]
            if r.get("kernel") == kernel:
                out.append(f"* the same run's bench line: dominant kernel {kernel}, "
                           f"{r['launches']} instrumented launches, avg_launch_ms "
                           f"{r['avg_launch_ms']} (HIP events)")
            elif kernel in bench.get("step_kernels", {}):
                a = bench["step_kernels"][kernel]["all"]
                out.append(f"* the same run's bench line: {a['launches']} instrumented launches, "
                           f"{a['ms']} ms in all, avg {a['ms'] / max(a['launches'], 1):.4f} ms "
                           f"(HIP events)")
    d = [(t1 - t0) / 1e3 for name, t0, t1 in rows if short(name) == "k_sssp_step"]
    if d:
        work = [x for x in d if x > NOOP_US]
        out += ["", "## k_sssp_step", "",
                f"* dispatches: {len(d)}, of which {len(d) - len(work)} are steps queued past "
                f"the end or steps with little work (< {NOOP_US:.0f} us)",
                f"* the others: {len(work)}, average {sum(work) / max(len(work), 1):.2f} us, "
                f"longest {max(work, default=0.0):.1f} us, {sum(work) / 1e3:.1f} ms in all"]
        if bench and bench.get("sssp"):
            out.append(f"* the same run's bench line: {bench['sssp']}")
    out += csr_build_section(rows, short)
    print("\n".join(out))


def csr_build_section(rows, short):
    """The CSR build of the largest graph in a kernel trace: its kernels from
    the longest packing dispatch up to the first traversal after it."""
    packs = [(t1 - t0, t0) for name, t0, t1 in rows if short(name) == "k_pack"]
    if not packs:
        return []
    build = ("k_pack", "k_hist_reduce", "k_digit_starts", "k_onesweep", "k_scan_u32",
             "k_set_u64", "k_heads_count", "k_compact", "k_iso", "k_rp32", "k_find_hubs",
             "k_hub_", "k_deg16", "k_hint", "k_hot_", "k_chunk_count")
    is_build = lambda k: k.startswith(build)
    start = max(packs)[1]
    # up to the first other kernel of the library after the packing
    after = [t0 for name, t0, t1 in rows
             if t0 > start and short(name).startswith("k_") and not is_build(short(name))]
    stop = min(after) if after else float("inf")
    agg, last = {}, start
    for name, t0, t1 in rows:
        if start <= t0 < stop and is_build(short(name)):
            a = agg.setdefault(short(name), [0, 0.0])
            a[0] += 1
            a[1] += (t1 - t0) / 1e3
            last = max(last, t1)
    total = sum(a[1] for a in agg.values())
    out = ["", "## CSR build of the largest graph of the run", "",
           f"Kernel time {total / 1e3:.1f} ms; first kernel start to last kernel end "
           f"{(last - start) / 1e6:.1f} ms (the build's own kernels; its copies and fills "
           "and the host's reads of counts lie in between).", "",
           "| kernel | calls | total ms | % |", "|---|---:|---:|---:|"]
    for k, (n, t) in sorted(agg.items(), key=lambda kv: -kv[1][1]):
        if t >= 10.0:
            out.append(f"| `{k}` | {n} | {t / 1e3:.2f} | {100 * t / total:.1f} |")
    return out


def run_gpu(args):
    import torch
    import kronecker as K
    import paper_2012_13548_amd as g5

    dev = torch.device("cuda:0")
    scale, n = args.scale, 1 << args.scale
    # load every kernel once on a small graph
    small = g5.build_csr(K.edges_device(10, device=dev), 1 << 10)
    g5.bfs(small, 0)
    del small

    log(f"generating scale-{scale} ef{args.edgefactor} tuples on the device")
    edges = K.edges_device(scale, args.edgefactor, device=dev)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    csr = g5.build_csr(edges, n)
    e1.record()
    torch.cuda.synchronize()
    build_ms = e0.elapsed_time(e1)
    log(f"g5_build_csr: nnz {csr.nnz} in {build_ms:.1f} ms")
    mask = K.nonisolated_device(edges, n).cpu().numpy()
    roots = K.select_roots(mask, args.roots, K.root_seed(scale))
    del edges, mask
    torch.cuda.empty_cache()

    rp, _ = csr.arrays()
    deg = (rp[1:] - rp[:-1])
    del rp
    parent = torch.empty(n, dtype=torch.int32, device=dev)
    level = torch.empty(n, dtype=torch.int32, device=dev)

    # Untimed accounting pass: traversed edges m_r, the library's own byte
    # count per level (count_bytes), and the work counts of every level from
    # the finished level array (g5_level_work), which give the algorithmic
    # bytes of each step by the definition in include/g5.h.
    m_r, acct, work = [], [], []
    for r in roots:
        _, _, st = g5.bfs(csr, r, parent, level, count_bytes=True)
        m_r.append(int(deg[level >= 0].sum().item()) // 2)
        acct.append(st)
        work.append([g5.level_work(csr, level, lv, bottom_up=st["dir"][lv] == 2)
                     if lv < len(st["dir"]) else g5.level_work(csr, level, lv)
                     for lv in range(st["nlevels"])])
    del deg
    log(f"accounting done: m_r of root 0 = {m_r[0]}, levels {acct[0]['nlevels']}, "
        f"dirs {acct[0]['dir']}")

    for _ in range(args.warmup):
        for r in roots:
            g5.bfs(csr, r, parent, level)
    torch.cuda.synchronize()
    log(f"warmup {args.warmup} step(s) done")

    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in roots]
    samples = []
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for step in range(args.steps):
        for i, r in enumerate(roots):
            ev[i][0].record()
            g5.bfs(csr, r, parent, level)
            ev[i][1].record()
        torch.cuda.synchronize()
        for i, r in enumerate(roots):
            samples.append(m_r[i] / (ev[i][0].elapsed_time(ev[i][1]) / 1e3))
        log(f"step {step + 1}/{args.steps}: hmean so far {hmean(samples) / 1e9:.2f} GTEPS")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start

    # Instrumented pass over the same roots, right after the timed steps: each
    # level's step kernel carries HIP start/stop events in its own dispatch on
    # the library's stream.  It is kept out of the timed steps because timed
    # dispatches slow the whole traversal by ~6 %.
    stats = [g5.bfs(csr, r, parent, level, time_steps=True)[2] for r in roots]
    # the run's last traversal is a plain one from the first root: counter
    # runs of this command read its levels in dispatch order
    g5.bfs(csr, roots[0], parent, level)
    torch.cuda.synchronize()
    steps = step_table(stats, acct, work, n)
    log(f"instrumented pass done: {len(steps)} step kernels timed")
    roofline, per_kernel = roofline_of(steps, scale)
    per_level = [{k: v for k, v in st.items() if k != "root"} for st in steps
                 if st["root"] == 0]
    # measured HBM bytes per level of the first root, from the counter runs
    lv_bytes = measured_traffic("root0_levels", f"s{scale}", "levels")
    if lv_bytes and [x["dir"] for x in lv_bytes] == [p["dir"] for p in per_level]:
        for p, x in zip(per_level, lv_bytes):
            p["hbm_bytes"] = x["bytes"]
            p["hbm_gbs"] = round(x["bytes"] / (p["ms"] / 1e3) / 1e9, 1) if p["ms"] else None
    gpu = {"value": hmean(samples) / 1e9, "ms_per_step": wall * 1e3 / args.steps,
           "build_ms": build_ms, "nnz": csr.nnz, "roots": roots, "m_r": m_r,
           "roofline": roofline, "steps": per_kernel, "per_level_root0": per_level}
    return gpu, csr, parent, level


def step_bytes(direction, w, n):
    """Algorithmic bytes of one step from its level's work counts (g5_level_work):
    top-down 20|Q| + 4 m_f + 12 claimed; bottom-up 16 U + 4 S + n/4 + 8 claimed."""
    if direction == 1:
        return 20 * w["q"] + 4 * w["mf"] + 12 * w["claimed"]
    return 16 * w["unvisited"] + 4 * w["scanned"] + n // 4 + 8 * w["claimed"]


def step_table(stats, acct, work, n):
    """One row per (root, level): its step kernel, device time (instrumented
    pass), algorithmic bytes, the library's own byte count, and its share of
    the traversal's edge work (top-down: frontier edges; bottom-up: row entries
    read up to the first frontier neighbour)."""
    rows = []
    for ri, (st, ac, wk) in enumerate(zip(stats, acct, work)):
        nl = min(st["nlevels"], len(st["dir"]), len(wk))
        edge = [wk[lv]["mf"] if st["dir"][lv] == 1 else wk[lv]["scanned"] for lv in range(nl)]
        total = max(sum(edge), 1)
        for lv in range(nl):
            d = st["dir"][lv]
            kernel = ("k_td_expand" if d == 1 else
                      "k_bu_step_lds" if (st["lds_mask"] >> lv) & 1 else "k_bu_step")
            b = step_bytes(d, wk[lv], n)
            ms = st["step_ms"][lv]
            rows.append({"root": ri, "level": lv, "dir": "TD" if d == 1 else "BU",
                         "kernel": kernel, "frontier": st["frontier"][lv],
                         "discovered": st["discovered"][lv], "edge_work": edge[lv],
                         "edge_share": round(edge[lv] / total, 4), "ms": round(ms, 4),
                         "alg_bytes": b,
                         "lib_bytes": ac["bytes"][lv] if ac["dir"][lv] == d else None,
                         "frac": round(b / (ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4) if ms else None})
    return rows


def roofline_of(steps, scale):
    """The dominant step kernel (largest total device time) against the HBM
    peak, with every step kernel's totals beside it, over all steps and over
    the steps that carry at least 1 % of their traversal's edge work."""
    agg = {}
    for st in steps:
        for key in ("all", "ge1pct"):
            if key == "ge1pct" and st["edge_share"] < 0.01:
                continue
            a = agg.setdefault(st["kernel"], {}).setdefault(
                key, {"launches": 0, "ms": 0.0, "alg_bytes": 0, "lib_bytes": 0})
            a["launches"] += 1
            a["ms"] += st["ms"]
            a["alg_bytes"] += st["alg_bytes"]
            a["lib_bytes"] += st["lib_bytes"] or 0
    per_kernel = {}
    for k, d in agg.items():
        per_kernel[k] = {}
        for key, a in d.items():
            gbs = a["alg_bytes"] / (a["ms"] / 1e3) / 1e9 if a["ms"] else 0.0
            lgbs = a["lib_bytes"] / (a["ms"] / 1e3) / 1e9 if a["ms"] else 0.0
            per_kernel[k][key] = {"launches": a["launches"], "ms": round(a["ms"], 3),
                                  "alg_gbs": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4),
                                  "lib_gbs": round(lgbs, 1),
                                  "lib_frac": round(lgbs / HBM_PEAK_GBS, 4)}
    dom = max(agg, key=lambda k: agg[k]["all"]["ms"])
    a = agg[dom]["all"]
    achieved = a["alg_bytes"] / (a["ms"] / 1e3) / 1e9
    total_ms = sum(x["all"]["ms"] for x in agg.values())
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": measured_traffic(dom, f"s{scale}"), "kernel": dom,
                "traffic_raw": measured_traffic(dom, f"s{scale}", "raw_bytes_per_launch"),
                "read_requests": measured_traffic(dom, f"s{scale}", "read_requests_per_launch"),
                "launches": a["launches"], "avg_launch_ms": round(a["ms"] / a["launches"], 4),
                "alg_bytes_per_launch": int(a["alg_bytes"] / a["launches"]),
                "time_share": round(a["ms"] / total_ms, 3),
                "lib_bytes_per_launch": int(a["lib_bytes"] / a["launches"]),
                "lib_frac": round(a["lib_bytes"] / (a["ms"] / 1e3) / 1e9 / HBM_PEAK_GBS, 4)}
    return roofline, per_kernel


def run_alg3_curve(args):
    """The host experiment's speedup curve: the paper's parallel level-synchronous
    BFS (OpenMP threads, libg5alg3.so) on a Kronecker graph built on the GPU and
    copied to the host, over thread counts up to this host's share (at most 16),
    a few roots each; one root's levels are checked against the GPU's."""
    import numpy as np
    import torch
    import kronecker as K
    import paper_2012_13548_amd as g5
    from paper_2012_13548_amd import alg3
    scale, n = args.alg3_scale, 1 << args.alg3_scale
    dev = torch.device("cuda:0")
    edges = K.edges_device(scale, args.edgefactor, device=dev)
    csr = g5.build_csr(edges, n)
    roots = K.select_roots(K.nonisolated_device(edges, n).cpu().numpy(), args.alg3_roots,
                           K.root_seed(scale))
    del edges
    _, gpu_level = g5.bfs(csr, roots[0])
    gpu_level = gpu_level.cpu().numpy()
    rp_t, ci_t = csr.arrays()
    rp, ci = rp_t.cpu().numpy(), ci_t.cpu().numpy()
    deg = np.diff(rp)
    cores = len(os.sched_getaffinity(0))
    threads = [t for t in (1, 2, 4, 8, 16) if t <= min(cores, 16)]
    rows, equal = [], True
    for t in threads:
        secs, teps = [], []
        for i, r in enumerate(roots):
            _, level, sec = alg3.bfs(rp, ci, r, t)
            if i == 0:
                equal = equal and bool(np.array_equal(level, gpu_level))
            secs.append(sec)
            teps.append((int(deg[level >= 0].sum()) // 2) / sec)
        rows.append({"threads": t, "mean_s": round(float(np.mean(secs)), 5),
                     "hmean_gteps": round(hmean(teps) / 1e9, 4)})
        log(f"alg3 threads {t}: {rows[-1]}")
    for row in rows:
        row["speedup"] = round(rows[0]["mean_s"] / row["mean_s"], 2)
    print(json.dumps({"alg3_curve": {"scale": scale, "edgefactor": args.edgefactor,
                                     "roots": len(roots), "host_threads": cores,
                                     "levels_equal_gpu": equal, "rows": rows}}))


def run_batch(args):
    """64 roots at scale 22: one batched launch vs 64 sequential single-root runs."""
    import torch
    import kronecker as K
    import paper_2012_13548_amd as g5
    dev = torch.device("cuda:0")
    scale, n = args.batch_scale, 1 << args.batch_scale
    edges = K.edges_device(scale, args.edgefactor, device=dev)
    csr = g5.build_csr(edges, n)
    mask = K.nonisolated_device(edges, n).cpu().numpy()
    roots = K.select_roots(mask, 64, K.root_seed(scale))
    del edges
    rp, _ = csr.arrays()
    deg = rp[1:] - rp[:-1]
    parent = torch.empty(n, dtype=torch.int32, device=dev)
    level = torch.empty(n, dtype=torch.int32, device=dev)
    m_r = []
    for r in roots:
        g5.bfs(csr, r, parent, level)
        m_r.append(int(deg[level >= 0].sum().item()) // 2)
    parents = torch.empty((64, n), dtype=torch.int32, device=dev)
    levels = torch.empty((64, n), dtype=torch.int8, device=dev)
    try:
        g5.bfs_batch(csr, roots, levels=levels, parent_out=parents)
    except g5.G5Error as e:
        log(f"batched BFS unavailable: {e}")
        return None
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 3
    seq, bat, bat_lv, bat_g = [], [], [], []
    g5.bfs_batch(csr, roots, levels=levels, parent_out=parents, graph=True)  # instantiate
    for _ in range(reps):
        torch.cuda.synchronize()
        e0.record()
        for r in roots:
            g5.bfs(csr, r, parent, level)
        e1.record()
        torch.cuda.synchronize()
        seq.append(e0.elapsed_time(e1) / 1e3)
        e0.record()
        g5.bfs_batch(csr, roots, levels=levels, parent_out=parents)
        e1.record()
        torch.cuda.synchronize()
        bat.append(e0.elapsed_time(e1) / 1e3)
        e0.record()
        g5.bfs_batch(csr, roots, parents=False, levels=levels)
        e1.record()
        torch.cuda.synchronize()
        bat_lv.append(e0.elapsed_time(e1) / 1e3)
        e0.record()
        g5.bfs_batch(csr, roots, levels=levels, parent_out=parents, graph=True)
        e1.record()
        torch.cuda.synchronize()
        bat_g.append(e0.elapsed_time(e1) / 1e3)
    total = sum(m_r)
    t_seq, t_bat, t_lv = min(seq), min(bat), min(bat_lv)
    return {"scale": scale, "roots": 64, "with_parents": True,
            "sequential_gteps": round(total / t_seq / 1e9, 3),
            "batched_gteps": round(total / t_bat / 1e9, 3),
            "ratio": round(t_seq / t_bat, 3), "sequential_ms": round(t_seq * 1e3, 3),
            "batched_ms": round(t_bat * 1e3, 3),
            "levels_only": {"batched_ms": round(t_lv * 1e3, 3),
                            "batched_gteps": round(total / t_lv / 1e9, 3),
                            "ratio": round(t_seq / t_lv, 3)},
            "graph_replays": {"batched_ms": round(min(bat_g) * 1e3, 3),
                              "ratio": round(t_seq / min(bat_g), 3)}}


def run_sssp(args):
    """Kernel 3 (SSSP by delta-stepping) on a weighted Kronecker graph: per
    root, device time of g5_sssp (events around the call) and m_r, the
    distinct edges of the root's component; harmonic mean of m_r / t over the
    roots.  The first root's distances are checked against the oracle's
    Dijkstra when --sssp-oracle is given."""
    import numpy as np
    import torch
    import kronecker as K
    import paper_2012_13548_amd as g5
    dev = torch.device("cuda:0")
    scale, n = args.sssp_scale, 1 << args.sssp_scale
    edges = K.edges_device(scale, args.edgefactor, device=dev)
    weights = K.weights_device(scale, args.edgefactor, device=dev)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    csr = g5.build_csr_w(edges, weights, n)
    e1.record()
    torch.cuda.synchronize()
    build_ms = e0.elapsed_time(e1)
    roots = K.select_roots(K.nonisolated_device(edges, n).cpu().numpy(), args.sssp_roots,
                           K.root_seed(scale))
    del edges, weights
    rp, _ = csr.arrays()
    deg = rp[1:] - rp[:-1]
    dist = torch.empty(n, dtype=torch.int32, device=dev)
    prev = torch.empty(n, dtype=torch.int32, device=dev)
    m_r, infos = [], []
    for r in roots:
        _, _, info = g5.sssp(csr, r, dist, prev, delta=args.sssp_delta, stats=True,
                             pull_div=args.sssp_pull_div)
        m_r.append(int(deg[dist != -1].sum().item()) // 2)
        infos.append(info)
    times = []
    for i, r in enumerate(roots):
        e0.record()
        g5.sssp(csr, r, dist, prev, delta=args.sssp_delta, pull_div=args.sssp_pull_div)
        e1.record()
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1) / 1e3)
    teps = [m / t for m, t in zip(m_r, times)]
    out = {"scale": scale, "roots": len(roots), "weights": "integers 1..255 per tuple",
           "delta": infos[0]["delta"], "hmean_gteps": round(hmean(teps) / 1e9, 3),
           "mean_ms": round(1e3 * sum(times) / len(times), 3), "csr_build_ms": round(build_ms, 2),
           "mean_rounds": round(sum(i["rounds"] for i in infos) / len(infos), 1),
           "mean_buckets": round(sum(i["buckets"] for i in infos) / len(infos), 1),
           "mean_pulls": round(sum(i["pulls"] for i in infos) / len(infos), 1)}
    if args.sssp_oracle:
        import oracle as O
        eh, wh = K.edges_host(scale, args.edgefactor), K.weights_host(scale, args.edgefactor)
        ocsr = O.build_csr_w(eh, wh, n)
        del eh, wh
        g5.sssp(csr, roots[0], dist, prev, delta=args.sssp_delta, pull_div=args.sssp_pull_div)
        od, _, dt = O.sssp_timed(ocsr, roots[0])
        out["oracle_root0_s"] = round(dt, 3)
        out["oracle_root0_gteps"] = round(m_r[0] / dt / 1e9, 5)
        gd = dist.cpu().numpy().view(np.uint32)
        out["dist_equal_oracle"] = bool(np.array_equal(gd, od))
        out["prev_equal_oracle"] = bool(np.array_equal(prev.cpu().numpy(),
                                                       O.min_prev(ocsr, roots[0], od)))
    return out


def run_serve(args):
    """Serving extra: BFS requests on graphs of scales 16, 18, 20, 22 and 23
    resident at once, Poisson arrivals at 0.7 of the saturated rate; latency
    is completion minus arrival per request."""
    from paper_2012_13548_amd import serve as S
    out = S.run_poisson(requests=args.serve_requests, log=lambda m: log(f"serve: {m}"))
    keep = ("requests", "errors", "error_kinds", "p50_ms", "p99_ms", "mean_ms", "throughput_rps",
            "aggregate_gteps", "mean_batch", "rate_rps", "saturated_rps", "load", "scales",
            "workers")
    return {k: out[k] for k in keep}


def host_threads():
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count() or 1


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return ""


def run_cpu(args, roots, gpu_level_of):
    """The oracle timed on this host's cores: its single-threaded queue BFS from
    every root of the same graph, on its own CSR built from the host generator
    (build untimed), roots spread over P worker threads (P = this host's share
    of cores, capped by what fits in memory; each call holds its queue, level
    and parent arrays).  Each root's oracle levels are compared with the GPU's
    (gpu_level_of(root) -> numpy int32 levels)."""
    from concurrent.futures import ThreadPoolExecutor
    import numpy as np
    import kronecker as K
    import oracle as O
    scale, n = args.scale, 1 << args.scale
    log("cpu baseline: host generator")
    edges = K.edges_host(scale, args.edgefactor)
    log("cpu baseline: oracle CSR")
    ocsr = O.build_csr(edges, n)
    del edges
    roots = roots[:args.cpu_roots]
    per_root = 12 * n  # queue, level and parent arrays of one oracle call
    try:
        import psutil
        avail = psutil.virtual_memory().available
    except ImportError:
        avail = 64 << 30
    P = max(1, min(host_threads(), args.cpu_threads or 10 ** 6, len(roots),
                   int(0.6 * avail // per_root)))
    log(f"cpu baseline: {len(roots)} roots on {P} threads")

    def one(r):
        _, lev, dt = O.bfs_timed(ocsr, r)
        return lev, dt

    secs, teps, mrs, equal = [], [], [], 0
    t0 = time.perf_counter()
    with ThreadPoolExecutor(P) as ex:
        for r, (lev, dt) in zip(roots, ex.map(one, roots)):
            mr = O.teps_edges(ocsr, lev)
            secs.append(dt)
            mrs.append(mr)
            teps.append(mr / dt)
            equal += int(np.array_equal(lev, gpu_level_of(r)))
            log(f"cpu baseline: root {r}: {dt:.2f} s, {mr / dt / 1e6:.1f} MTEPS")
    wall = time.perf_counter() - t0
    return {"value": round(hmean(teps) / 1e9, 5), "unit": "GTEPS", "cores": P,
            "kind": "oracle",
            "sample": f"single-threaded oracle queue BFS from each of {len(roots)} roots of the "
                      f"same scale-{scale} graph, {P} at a time on {P} host threads "
                      f"({sum(secs):.1f} s of BFS in {wall:.1f} s wall); value = harmonic mean "
                      f"of per-root TEPS (one core per root); oracle's own CSR from the host "
                      f"generator, build untimed",
            "per_root_s": [round(x, 3) for x in secs],
            "wall_s": round(wall, 2),
            "aggregate_gteps": round(sum(mrs) / wall / 1e9, 5),
            "host_cpu": cpu_model(), "host_threads": host_threads(),
            "levels_equal_gpu": f"{equal}/{len(roots)}"}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--scale", type=int, default=26)
    ap.add_argument("--edgefactor", type=int, default=16)
    ap.add_argument("--roots", type=int, default=64)
    ap.add_argument("--batch-scale", type=int, default=22)
    ap.add_argument("--cpu-roots", type=int, default=64,
                    help="roots of the CPU oracle baseline (default: all 64)")
    ap.add_argument("--cpu-threads", type=int, default=0,
                    help="oracle worker threads (default: this host's share of cores)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-sssp", action="store_true")
    ap.add_argument("--sssp-scale", type=int, default=22)
    ap.add_argument("--sssp-roots", type=int, default=16)
    ap.add_argument("--sssp-delta", type=int, default=0)
    ap.add_argument("--sssp-pull-div", type=int, default=0,
                    help="SSSP rounds with at least nnz/this many edges pull (0: default, <0: never)")
    ap.add_argument("--sssp-oracle", action="store_true",
                    help="check the first SSSP root against the oracle's Dijkstra (slow)")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=2000,
                    help="Poisson requests of the serving extra (graphs of scales 16-23 resident)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="run the counter-calibration copy kernel first")
    ap.add_argument("--gather-probe", action="store_true",
                    help="run the random-gather calibration kernel first")
    ap.add_argument("--reduce-pmc", nargs="+", metavar="DIR",
                    help="write profiles/traffic.json from rocprofv3 --pmc runs (FETCH_SIZE dir, "
                         "WRITE_SIZE dir, optionally the request-split dir) and exit")
    ap.add_argument("--pmc-command", default="", help="command recorded with --reduce-pmc")
    ap.add_argument("--summarize-trace", nargs="+", metavar=("DB", "BENCH_JSON"),
                    help="print a markdown summary of a rocprofv3 kernel-trace database")
    ap.add_argument("--trace-command", default="", help="command recorded with --summarize-trace")
    ap.add_argument("--trace-title", default="", help="heading of the --summarize-trace summary")
    ap.add_argument("--alg3-curve", action="store_true",
                    help="time the host experiment (the paper's parallel level-synchronous BFS "
                         "with OpenMP) over thread counts, print one JSON line and exit")
    ap.add_argument("--alg3-scale", type=int, default=20)
    ap.add_argument("--alg3-roots", type=int, default=4)
    args = ap.parse_args()
    if args.alg3_curve:
        run_alg3_curve(args)
        return
    if args.summarize_trace:
        summarize_trace(args.summarize_trace[0], args.trace_command,
                        args.summarize_trace[1] if len(args.summarize_trace) > 1 else None,
                        **({"title": args.trace_title} if args.trace_title else {}))
        return
    if args.reduce_pmc:
        reduce_pmc(args.reduce_pmc[0], args.reduce_pmc[1],
                   args.reduce_pmc[2] if len(args.reduce_pmc) > 2 else None, f"s{args.scale}",
                   args.pmc_command)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the many-root workload shards by roots with no communication: run one "
              "process per GPU instead)", file=sys.stderr)
        sys.exit(2)

    if args.copy_probe:
        copy_probe()
    if args.gather_probe:
        gather_probe()
    gpu, csr, parent, level = run_gpu(args)
    import torch
    import paper_2012_13548_amd as g5
    batch = None if args.no_batch else run_batch(args)
    if batch:
        log(f"batch: ratio {batch['ratio']} ({batch['batched_gteps']} vs "
            f"{batch['sequential_gteps']} GTEPS)")
    sssp = None if args.no_sssp else run_sssp(args)
    if sssp:
        log(f"sssp: {sssp}")
    serve = None if args.no_serve else run_serve(args)
    if serve:
        log(f"serve: {serve}")
    cpu = None
    if not args.no_cpu:
        def gpu_level_of(r):
            g5.bfs(csr, r, parent, level)
            return level.cpu().numpy()
        cpu = run_cpu(args, gpu["roots"], gpu_level_of)
    del csr, parent, level
    torch.cuda.empty_cache()

    out = {
        "metric": METRIC,
        "value": round(gpu["value"], 3),
        "unit": "GTEPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(gpu["ms_per_step"], 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": f"kronecker-scale{args.scale}-ef{args.edgefactor}-"
                               f"{args.roots}roots-single-root-bfs",
                   "scale": args.scale, "edgefactor": args.edgefactor,
                   "vertices": 1 << args.scale, "tuples": args.edgefactor << args.scale,
                   "nnz": gpu["nnz"], "roots": args.roots,
                   "generator": "seeded Kronecker (0.57,0.19,0.19,0.05), relabelled, "
                                "graph seed 1000+scale, root seed 2000+scale"},
        "roofline": gpu["roofline"],
        "cpu_baseline": cpu,
        "csr_build_ms": round(gpu["build_ms"], 2),
        "batch": batch,
        "sssp": sssp,
        "serve": serve,
        "step_kernels": gpu["steps"],
        "per_level_root0": gpu["per_level_root0"],
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
