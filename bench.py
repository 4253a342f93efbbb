#!/usr/bin/env python3
"""Benchmark of the Manifold k-NN query path on one MI355X.

A step is one pass of the whole query path over one batch: the query batch preparation
(Morton bucketing), the 1-NN descent (Alg. 1) and the k-expansion (Alg. 2) with the prefix
bound, writing indices and distances -- for the headline workload: 1,000,000 points on a
torus (R=1, r=0.3, normal noise 1e-3, random insertion order), 1,000,000 volume queries
uniform in the bounding box expanded by 10%, k=16, m=n.  Inputs are resident in HBM
before timing starts; the host-side list construction is reported but not timed.

The default run also measures, for the same JSON line: the memory probes (streaming read
and random 16-byte gathers), the FP64 brute-force oracle on the host cores with the parity
of the rows it computed, and -- in a child process started before this one touches the
GPU, so that each process's kernel statistics stay separate under a profiler -- the
batched form (256 clouds, one launch per class against one plain launch per cloud) and
the serving form (64 resident clouds, continuous batching against one launch per request:
saturation, p50/p99 in an open loop with deletions, a sweep of offered loads), each
checked against the oracle.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import collections
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E, published
METRIC = "k-NN queries/sec (k=16, 1M-pt surface) + p50/p99 latency, batched vs plain"


_T0 = time.perf_counter()


def log(msg: str) -> None:
    print(f"[bench {time.perf_counter() - _T0:7.1f}s] {msg}", file=sys.stderr, flush=True)


# the query kernel of the headline workload: one slot per lane (k <= 16), k == 16 exactly,
# descent steps first, one k and m per launch, no pending-deletion filter
HEADLINE_KERNEL = "knn_rows_kernel<1, true, true, true, false>"

# the translation unit of the plain query path and the headers its kernels are built from
KERNEL_SOURCES = ("mknn_device.hip", "knn_kernels.h", "knn_group.h", "knn_rows.h",
                  "device_common.h", "planefit.h")


def csrc_digest() -> str:
    """Hash of the sources the plain query kernels are compiled from, to tell whether stored
    counter readings still apply (host-only code, the batched and serving translation units
    and the probes do not enter)."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2605_02224_amd", "csrc")
    for f in KERNEL_SOURCES:
        h.update(f.encode())
        h.update(open(os.path.join(csrc, f), "rb").read())
    return h.hexdigest()


def measured_traffic(k: int):
    """HBM bytes per launch of the query kernel from the committed rocprofv3 readings
    (FETCH_SIZE and WRITE_SIZE, scaled by a plain copy kernel), or None once the kernel
    sources changed since those counters were taken."""
    path = os.path.join(ROOT, "profiles", "knn_traffic.json")
    if k != 16 or not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("csrc_sha256") != csrc_digest():
        return None
    return rec.get("traffic_bytes_per_dispatch")


def ingest_counters(fetch_dir: str, write_dir: str, out_path: str, last: int) -> dict:
    """Write the HBM byte reading of the headline query kernel from two rocprofv3 --pmc runs
    of this benchmark with --copy-probe (FETCH_SIZE in one, WRITE_SIZE in the other):
    KiB per dispatch over the last `last` dispatches of the kernel (the timed steps; the
    autotuner's and the warm-up's launches come before them), each scaled by what the same
    counter reads for the copy probe (an elementwise pass reading and writing 1 GiB),
    stamped with the hash of the kernel sources the counters were taken from."""
    import csv
    import glob
    kname = HEADLINE_KERNEL
    probe = "elementwise_kernel"
    rec = {"kernel": "mknn::" + kname, "workload": "torus 1M points, 1M volume queries, k=16, m=n",
           "csrc_sha256": csrc_digest()}
    for counter, d in (("FETCH_SIZE", fetch_dir), ("WRITE_SIZE", write_dir)):
        kern, copy = [], []
        for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
            for i, row in enumerate(csv.DictReader(open(f))):
                if row.get("Counter_Name") != counter:
                    continue
                name = row.get("Kernel_Name", "")
                if kname in name:
                    kern.append((int(row.get("Dispatch_Id") or 0), i, float(row["Counter_Value"])))
                elif probe in name:
                    copy.append(float(row["Counter_Value"]))
        if not kern or not copy:
            raise RuntimeError(f"{counter}: no dispatch of the query kernel or the copy probe "
                               f"under {d}")
        kern = [v for _, _, v in sorted(kern)][-last:]
        key = "fetch" if counter == "FETCH_SIZE" else "write"
        rec[f"{key}_kib_per_dispatch"] = round(sum(kern) / len(kern), 1)
        rec[f"{key}_dispatches"] = len(kern)
        # the probe is the largest elementwise pass of the run (1 GiB in, 1 GiB out); the
        # benchmark's other elementwise kernels are small conversions and reductions
        rec[f"{key}_probe_kib"] = max(copy)
        rec[f"{key}_scale"] = round((1 << 20) / max(copy), 4)
    rec["traffic_bytes_per_dispatch"] = 1024.0 * (
        rec["fetch_kib_per_dispatch"] * rec["fetch_scale"] +
        rec["write_kib_per_dispatch"] * rec["write_scale"])
    with open(out_path, "w") as f:
        json.dump(rec, f, indent=2)
    return rec


def trace_summary(trace_dir: str, last: int) -> dict:
    """Durations of the headline query kernel in rocprofv3 kernel-trace CSVs of this
    benchmark (one file per process): the dispatches of the headline kernel
    over the 1M-query grid in launch order, and the mean of the last `last` of them (the
    timed steps of a run with --no-extras)."""
    import csv
    import glob
    out = {}
    for f in sorted(glob.glob(os.path.join(trace_dir, "**", "*kernel_trace.csv"), recursive=True)):
        durs = []
        for r in csv.DictReader(open(f)):
            if HEADLINE_KERNEL not in r.get("Kernel_Name", ""):
                continue
            grid = int(r.get("Grid_Size") or r.get("Grid_Size_X") or 0)
            durs.append((int(r["Start_Timestamp"]), grid,
                         (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e6))
        big = [d for _, g, d in sorted(durs) if g >= 16_000_000]
        if big:
            tail = big[-last:]
            out[os.path.basename(f)] = {
                "dispatches": len(durs), "headline_grid_dispatches": len(big),
                "timed_dispatches": len(tail),
                "timed_mean_ms": round(sum(tail) / len(tail), 4),
                "timed_ms": [round(d, 4) for d in tail]}
    return out


def cpu_info() -> dict:
    """Host CPU model and the cores this process may run on."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"model": model, "affinity_cpus": len(os.sched_getaffinity(0))}


def oracle_threads() -> int:
    """Threads for the oracle: the host cores available to the process, capped by the
    OMP_NUM_THREADS share when it is set."""
    n = len(os.sched_getaffinity(0))
    omp = os.environ.get("OMP_NUM_THREADS", "")
    if omp.isdigit() and int(omp) > 0:
        n = min(n, int(omp))
    return max(1, n)


def _time_oracle(P, Q, k, threads, target_s):
    """Oracle rows for a prefix of Q sized for about target_s of work on `threads` threads:
    (queries, seconds, idx, D)."""
    import oracle
    oracle.knn_bruteforce(P, Q[:16], k, threads=threads)       # load, start the threads
    n0 = min(64, Q.shape[0])
    while True:
        t = time.perf_counter()
        oracle.knn_bruteforce(P, Q[:n0], k, threads=threads)
        dt = max(time.perf_counter() - t, 1e-6)
        if dt >= 0.5 or n0 >= Q.shape[0]:
            break
        n0 = min(Q.shape[0], n0 * 4)
    ns = int(min(Q.shape[0], max(n0, n0 * target_s / dt)))
    t = time.perf_counter()
    idx, _, D = oracle.knn_bruteforce(P, Q[:ns], k, threads=threads)
    return ns, time.perf_counter() - t, idx, D


def cpu_baseline(P, Q, k, target_s: float, gpu_idx=None, gpu_dist=None):
    """Time the FP64 brute-force oracle on a bounded sample of the same queries (all
    allowed host cores, then one thread), and check the GPU rows of that sample against the
    rows the oracle computed.  Returns (baseline dict, parity dict or None)."""
    import oracle
    oracle.build(force=False)
    threads = oracle_threads()
    ns, dt, idx, D = _time_oracle(P, Q, k, threads, target_s)
    ns1, dt1, _, _ = _time_oracle(P, Q, k, 1, target_s / 4)
    info = cpu_info()
    base = {"value": ns / dt, "unit": "queries/s", "cores": threads, "kind": "oracle",
            "sample": f"first {ns} of the {Q.shape[0]} timed queries, brute force over all "
                      f"{P.shape[0]} points, FP64, {dt:.1f} s wall on {threads} threads; "
                      f"one thread: {ns1 / dt1:.1f} queries/s on the first {ns1}",
            "single_thread_qps": round(ns1 / dt1, 2), "cpu_model": info["model"],
            "affinity_cpus": info["affinity_cpus"]}
    parity = None
    if gpu_idx is not None:
        sys.path.insert(0, os.path.join(ROOT, "tests"))
        from _compare import compare_rows
        ties = compare_rows(gpu_idx[:ns], gpu_dist[:ns], idx, D, P=P, Q=Q[:ns])
        parity = {"rows": int(ns), "near_ties": int(ties), "mismatches": 0,
                  "oracle": "FP64 brute force, rows of the cpu_baseline sample"}
    return base, parity


def memory_probes() -> dict:
    """Measured memory rates on a 2 GiB buffer (larger than the 256 MB last-level cache):
    a streaming read and random 16-byte gathers."""
    import ctypes
    import torch
    from paper_2605_02224_amd import _lib
    L = _lib.lib()
    nbytes = 1 << 31
    buf = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    s = torch.cuda.current_stream().cuda_stream
    g = ctypes.c_double()
    _lib.check(L.mknn_probe_stream_read(buf.data_ptr(), nbytes, 5, s, ctypes.byref(g)))
    stream = g.value
    _lib.check(L.mknn_probe_gather16(buf.data_ptr(), nbytes, 1 << 27, 5, s, ctypes.byref(g)))
    gather = g.value
    del buf
    return {"stream_read_GBps": round(stream, 1), "gather16_GBps": round(gather, 1),
            "buffer_bytes": nbytes}


LAYOUTS = {"ranks": 1, "arrays": 2}   # MKNN_LAYOUT_RANKS, MKNN_LAYOUT_ARRAYS


def layout_probe(cl, q, idx, dist, records_ms: float, reps: int, k: int):
    """The same k=16 walk over two other layouts of the lists beside the record layout
    (coordinates inlined in 16-byte records): ranks only (a 4-byte rank per entry, the point
    gathered by rank) and four arrays (rank, x, y, z, 4 bytes each): kernel time of each, and
    whether the rows are bit-identical to the records' rows."""
    import ctypes
    import torch
    from paper_2605_02224_amd import _lib
    if k != 16:
        return None
    lib = _lib.lib()
    out = {"records_kernel_ms": round(records_ms, 4)}
    equal = True
    for name, layout in LAYOUTS.items():
        gi = torch.empty_like(idx)
        gd = torch.empty_like(dist)
        st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
        args = (cl.handle, layout, ctypes.c_void_p(q.data_ptr()), q.shape[0],
                ctypes.c_void_p(gi.data_ptr()), ctypes.c_void_p(gd.data_ptr()), st)
        for _ in range(2):
            _lib.check(lib.mknn_knn_layout(*args))
        torch.cuda.synchronize()
        tot = ctypes.c_double()
        cnt = ctypes.c_int64()
        lib.mknn_timing_enable(1)
        lib.mknn_timing_read(ctypes.byref(tot), ctypes.byref(cnt))   # reset
        for _ in range(max(3, reps // 4)):
            _lib.check(lib.mknn_knn_layout(*args))
        torch.cuda.synchronize()
        _lib.check(lib.mknn_timing_read(ctypes.byref(tot), ctypes.byref(cnt)))
        lib.mknn_timing_enable(0)
        ms = tot.value / max(cnt.value, 1)
        out[name + "_kernel_ms"] = round(ms, 4)
        out[name + "_slowdown"] = round(ms / records_ms, 3)
        equal = equal and bool(torch.equal(gi, idx) and torch.equal(gd, dist))
        del gi, gd
    out["rows_equal"] = equal
    return out


def build_clouds(clouds, threads: int = 16):
    """Build and upload many clouds: the lists are built on the GPU one cloud after the
    other (the same lists as the host construction, which the GPU tests check)."""
    from paper_2605_02224_amd.api import Cloud
    built = [Cloud.build(c.by_rank, device=True) for c in clouds]
    for c in built:
        c.upload()
    return built


def run_batched(args) -> dict:
    """Many clouds (sizes log-uniform in [1e3, 2e5], sphere/torus/ellipsoid, 4 n_c queries
    each, k=10): one flat launch per class and batch versus one plain launch per cloud; a
    sample of every cloud's rows checked against the oracle."""
    import torch
    from paper_2605_02224_amd import workloads as W
    from paper_2605_02224_amd import api as A
    t0 = time.perf_counter()
    w = W.many_clouds(num=args.clouds)
    npts = int(sum(c.n for c in w.clouds))
    log(f"batched: {len(w.clouds)} clouds, {npts} points generated in "
        f"{time.perf_counter() - t0:.1f} s")
    t0 = time.perf_counter()
    clouds = build_clouds(w.clouds, oracle_threads())
    build_s = time.perf_counter() - t0
    log(f"batched: built and uploaded in {build_s:.1f} s")
    qs = [torch.from_numpy(q).cuda() for q in w.queries]
    nq = sum(q.shape[0] for q in qs)
    items = A.alloc_outputs([(c, q, w.k, None) for c, q in zip(clouds, qs)])
    plan = A.BatchPlan(len(items), nq, tile_queries=args.tile, sort=True, graph=True)
    os.environ["MKNN_BATCH_PERSISTENT"] = "1"     # read at plan creation
    try:
        pplan = A.BatchPlan(len(items), nq, tile_queries=args.tile, sort=True, graph=True)
    finally:
        os.environ.pop("MKNN_BATCH_PERSISTENT", None)
    tuned = ptuned = None
    if not args.no_autotune:
        tuned = plan.tune(items)     # untimed: merge threshold of the flat launch
        ptuned = pplan.tune(items)   # untimed: tile length of the persistent launch
        log(f"batched: autotuner chose merge threshold {tuned} (flat), tile {ptuned} "
            f"(persistent)")
    torch.cuda.synchronize()

    def run_batch():
        plan.run(items)

    def run_persistent():
        pplan.run(items)

    def run_plain():
        for cl, q, k, m, idx, dist in items:
            cl.knn(q, k, out=(idx, dist))

    res = {}
    for name, fn in (("plain", run_plain), ("persistent", run_persistent),
                     ("batched", run_batch)):
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            fn()
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / args.steps
        res[name] = (nq / dt, dt)
        log(f"batched: {name} {nq / dt / 1e6:.1f} M queries/s, {dt * 1e3:.2f} ms per batch")
    # algorithmic bytes of the batch (untimed), by the headline's measure: 16 B per list entry
    # examined, 8 B per list opened, 12 B per query, 8 B per neighbour, from every query's
    # work counts
    tot_e = tot_l = 0
    for cl, q, k, m, idx, dist in items:
        ce, cn = cl.knn_counts(q, k)
        tot_e += int(ce.sum().item())
        tot_l += int(cn.sum().item())
    batch_bytes = 16 * tot_e + 8 * tot_l + (12 + 8 * w.k) * int(nq)
    frac = {name: round(batch_bytes / res[name][1] / (HBM_PEAK_GBS * 1e9), 4) for name in res}
    log(f"batched: {batch_bytes / 1e9:.2f} algorithmic GB per batch, roofline fraction "
        f"(step basis) {frac}")
    # parity of the last batched run: 256 sampled rows of every cloud
    import oracle
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    from _compare import compare_rows
    rng = np.random.default_rng(5)
    ties = rows = 0
    thr = oracle_threads()
    for c, (cl, q, k, m, idx, dist) in zip(w.clouds, items):
        Qa = q.cpu().numpy()
        sel = rng.choice(Qa.shape[0], min(256, Qa.shape[0]), replace=False)
        ri, _, rD = oracle.knn_bruteforce(c.by_rank, Qa[sel], k, threads=thr)
        ties += compare_rows(idx.cpu().numpy()[sel], dist.cpu().numpy()[sel], ri, rD,
                             P=c.by_rank, Q=Qa[sel])
        rows += sel.size
    log(f"batched: parity {rows} rows, {ties} near-tie positions")
    plan.close()
    pplan.close()
    return {"workload": f"batched_{len(items)}_clouds_k{w.k}", "clouds": len(items),
            "points": npts, "queries": int(nq), "k": w.k,
            "batched_qps": round(res["batched"][0], 1),
            "batched_ms": round(res["batched"][1] * 1e3, 3),
            "plain_qps": round(res["plain"][0], 1), "plain_ms": round(res["plain"][1] * 1e3, 3),
            "speedup_vs_plain": round(res["batched"][0] / res["plain"][0], 3),
            "persistent_qps": round(res["persistent"][0], 1),
            "persistent_ms": round(res["persistent"][1] * 1e3, 3),
            "form": "one flat launch per register class, hipGraph replay (the persistent "
                    "work-stealing launch beside it)",
            "merge_min_tuned": tuned, "persistent_tile_tuned": ptuned,
            "algorithmic_bytes_per_batch": int(batch_bytes),
            "entries_per_query": round(tot_e / nq, 2), "lists_per_query": round(tot_l / nq, 3),
            "roofline_frac_step_basis": frac,
            "build_s": round(build_s, 2),
            "parity": {"rows": rows, "near_ties": int(ties), "mismatches": 0}}


def bench_batched(args) -> int:
    r = run_batched(args)
    line = {
        "metric": METRIC, "value": r["batched_qps"], "unit": "queries/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": r["batched_ms"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": r["workload"], "clouds": r["clouds"], "points": r["points"],
                   "queries": r["queries"], "k": r["k"], "form": r["form"]},
        "extra": r,
    }
    print(json.dumps(line), flush=True)
    return 0


class _ServeRun:
    """One serving run: a submitter (this thread) feeds requests and deletion batches to an
    mknn server at scheduled times; a collector thread waits for them in order.  Request
    outputs live in a ring arena of device and pinned host buffers whose regions are reused
    once the request holding them has been collected."""

    def __init__(self, reqs, qoff, qd, ring, clouds):
        import ctypes
        from paper_2605_02224_amd import _lib
        self.L = _lib.lib()
        self.reqs = reqs
        d_idx, d_dist, h_idx, h_dist = ring
        self.h_idx, self.h_dist = h_idx, h_dist
        cap = d_idx.numel()
        # ring layout: requests take consecutive regions of an unbounded stream of positions
        # (skipping to the next multiple of the capacity rather than splitting a region);
        # physical position = stream position mod capacity.  Request i may start once every
        # request whose region starts less than one capacity before i's end is collected.
        sz = np.array([r.queries.shape[0] * r.k for r in reqs], np.int64)
        a = np.zeros(len(reqs), np.int64)
        pos = 0
        for i in range(len(reqs)):
            if pos % cap + sz[i] > cap:
                pos = (pos // cap + 1) * cap
            a[i] = pos
            pos += sz[i]
        self.need = np.searchsorted(a, a + sz - cap, side="left")
        self.start = a % cap
        self.size = sz
        self.arr = (_lib.Request * len(reqs))()
        self.hptr = []
        for i, r in enumerate(reqs):
            a = self.arr[i]
            a.cloud = clouds[r.cloud].handle.value
            a.d_q = qd.data_ptr() + int(qoff[i]) * 12
            a.nq = r.queries.shape[0]
            a.k = r.k
            a.m = r.m
            a.d_idx = d_idx.data_ptr() + int(self.start[i]) * 4
            a.d_dist = d_dist.data_ptr() + int(self.start[i]) * 4
            self.hptr.append((ctypes.c_void_p(h_idx.data_ptr() + int(self.start[i]) * 4),
                              ctypes.c_void_p(h_dist.data_ptr() + int(self.start[i]) * 4)))
        self.ctypes = ctypes

    def run(self, srv, lo, hi, arrivals=None, deletions=(), clouds=None, label="",
            capture=()):
        """Requests lo..hi-1; arrivals: offsets in seconds from the start (None = as fast as
        the ring allows); deletions: (position, cloud, ranks) submitted just before the
        request at that position; capture: request indices whose host rows are copied out
        when they complete (self.captured[i] = (idx, dist, updates seen)).  Returns
        per-request latencies, completion times and the first scheduled arrival."""
        import queue
        import threading
        ct = self.ctypes
        L = self.L
        h = srv._h
        q = queue.Queue()
        n = hi - lo
        lat = np.zeros(n)
        t_done = np.zeros(n)
        t_wait = np.zeros(n)      # submitted -> launched
        t_lag = np.zeros(n)       # scheduled arrival -> submitted
        state = {"collected": lo, "err": None}
        cv = threading.Condition()
        capture = set(capture)
        self.captured = {}

        def collect():
            tt = (ct.c_double * 3)()
            v = ct.c_int64()
            while True:
                item = q.get()
                if item is None:
                    return
                i, tk, t_sched = item
                st = L.mknn_server_wait(h, ct.c_uint64(tk), tt, ct.byref(v))
                if st != 0 and state["err"] is None:
                    state["err"] = (i, st, L.mknn_last_error().decode())
                if i in capture:
                    a, b = int(self.start[i]), int(self.start[i] + self.size[i])
                    r = self.reqs[i]
                    self.captured[i] = (self.h_idx[a:b].numpy().reshape(-1, r.k).copy(),
                                        self.h_dist[a:b].numpy().reshape(-1, r.k).copy(),
                                        int(v.value))
                lat[i - lo] = tt[2] - t_sched
                t_done[i - lo] = tt[2]
                t_lag[i - lo] = tt[0] - t_sched
                t_wait[i - lo] = tt[1] - tt[0]
                with cv:
                    state["collected"] = i + 1
                    cv.notify_all()
                if (i - lo + 1) % 5000 == 0:
                    log(f"  {label}: {i - lo + 1}/{n} requests done")

        th = threading.Thread(target=collect, daemon=True)
        th.start()
        dels = sorted(deletions, key=lambda d: d[0])
        del_tickets = []   # waited for after the requests, so they never hold back the ring
        di = 0
        tk = ct.c_uint64()
        t0 = L.mknn_server_now() + 0.005
        t_first = None
        for i in range(lo, hi):
            while di < len(dels) and dels[di][0] <= i:
                _, ci, ranks = dels[di]
                r = np.ascontiguousarray(ranks, dtype=np.int32)
                st = L.mknn_server_delete(h, clouds[ci].handle, ct.c_void_p(r.ctypes.data),
                                          r.shape[0], ct.byref(tk))
                if st != 0:
                    raise RuntimeError(L.mknn_last_error().decode())
                del_tickets.append(tk.value)
                srv._keep[tk.value] = (r,)
                di += 1
            if state["collected"] < self.need[i]:
                with cv:
                    cv.wait_for(lambda: state["collected"] >= self.need[i])
            if arrivals is not None:
                t_sched = t0 + arrivals[i - lo]
                while True:
                    d = t_sched - L.mknn_server_now()
                    if d <= 0:
                        break
                    if d > 2e-4:
                        time.sleep(d - 1e-4)
            else:
                t_sched = L.mknn_server_now()
            if t_first is None:
                t_first = t_sched
            hp = self.hptr[i]
            st = L.mknn_server_submit(h, ct.byref(self.arr[i]), hp[0], hp[1], ct.byref(tk))
            if st != 0:
                raise RuntimeError(L.mknn_last_error().decode())
            q.put((i, tk.value, t_sched))
        q.put(None)
        th.join()
        tt = (ct.c_double * 3)()
        for tk_ in del_tickets:
            st = L.mknn_server_wait(h, ct.c_uint64(tk_), tt, None)
            if st != 0 and state["err"] is None:
                state["err"] = ("deletion", st, L.mknn_last_error().decode())
        if state["err"] is not None:
            raise RuntimeError(f"request {state['err']}")
        self.parts = (t_lag, t_wait)
        return lat, t_done, t_first


def _merge_plans(parts):
    """One deletion plan from several disjoint ones (batches interleaved, seeded)."""
    plan = [b for p in parts for b in p]
    order = np.random.default_rng(3).permutation(len(plan))
    return [plan[i] for i in order]


def run_serving(args) -> dict:
    """Serving: 64 resident clouds (sizes log-uniform in [1e4, 2e6], about 24M points),
    requests of 1..65536 queries (log-uniform), k in {4, 16, 64}, prefix m uniform in
    [n/10, n]; open-loop Poisson arrivals at 0.7x the plain server's saturation rate; 1% of
    the points deleted in batches of <= 1000 between requests.  The batched server
    (continuous batching on stream slots) against the plain one (one launch per request);
    200 seeded requests of the batched run checked against the oracle on the live set each
    one was answered on; then a sweep of offered loads."""
    import torch
    from paper_2605_02224_amd import workloads as W
    from paper_2605_02224_amd import api as A
    sys.setswitchinterval(2e-4)   # the submitter and the collector hand the GIL over quickly
    t0 = time.perf_counter()
    w = W.serving_clouds(num=args.serving_clouds, n_hi=args.serving_n_hi)
    npts = sum(c.n for c in w.clouds)
    log(f"serving: {len(w.clouds)} clouds, {npts} points generated in "
        f"{time.perf_counter() - t0:.1f} s")
    t0 = time.perf_counter()
    clouds = build_clouds(w.clouds, oracle_threads())
    build_s = time.perf_counter() - t0
    log(f"serving: built and uploaded in {build_s:.1f} s")
    nwarm, nmeas, nsat = args.warm_requests, args.requests, args.sat_requests
    loads = [float(x) for x in args.sweep_loads.split(",")] if args.sweep_loads else []
    nsw, nsw_warm = args.sweep_requests, max(1, args.sweep_requests // 10)
    total = nsat + nwarm + nmeas + (nsw + nsw_warm)
    t0 = time.perf_counter()
    reqs = [w.request() for _ in range(total)]
    log(f"serving: {total} requests generated in {time.perf_counter() - t0:.1f} s")
    qoff = np.zeros(total + 1, np.int64)
    qoff[1:] = np.cumsum([r.queries.shape[0] for r in reqs])
    qd = torch.from_numpy(np.concatenate([r.queries for r in reqs])).cuda()
    cap = 1 << 26
    ring = (torch.empty(cap, dtype=torch.int32, device="cuda"),
            torch.empty(cap, dtype=torch.float32, device="cuda"),
            torch.empty(cap, dtype=torch.int32).pin_memory(),
            torch.empty(cap, dtype=torch.float32).pin_memory())
    torch.cuda.synchronize()
    run = _ServeRun(reqs, qoff, qd, ring, clouds)
    log(f"serving: {int(qoff[-1])} queries resident, output ring of {cap} entries")
    nq_of = np.diff(qoff)
    pool = 1 << 22

    def server(plain, bind=True, max_wave=256, lazy=False):
        return A.Server(pool_queries=pool, nstreams=args.slots, max_wave_requests=max_wave,
                        plain=plain, bind_at_admission=bind, lazy_delete=lazy)

    # saturation: the first nsat requests as fast as the ring allows, no deletions
    sat = {}
    for name in ("plain", "batched"):
        srv = server(name == "plain")
        run.run(srv, 0, min(500, nsat), label=f"{name} warm-up")
        lat, t_done, t_first = run.run(srv, 0, nsat, label=f"{name} saturation")
        span = float(t_done.max() - t_first)
        w_, r_ = srv.stats()
        srv.close()
        sat[name] = float(nq_of[:nsat].sum() / span)
        log(f"serving: {name} saturation {sat[name] / 1e6:.1f} M queries/s "
            f"({nsat / span:.0f} requests/s, {r_ / max(w_, 1):.2f} requests per wave)")

    # deletion plans over disjoint rank sets: delete_frac per main run (ten parts each), a
    # tenth of it per sweep run; the lists are re-packed before each load of the sweep, so
    # its five runs stay well within the arena slack and no run re-packs a cloud
    nsweep_runs = 5 * len(loads)
    tenth = w.deletion_plan(frac=args.delete_frac / 10, batch=1000, parts=20 + nsweep_runs)
    main_plans = [_merge_plans(tenth[0:10]), _merge_plans(tenth[10:20])]
    rng = np.random.default_rng(11)

    def open_loop(name, lo, hi, warm, load, plan, plain, bind=True, max_wave=256, capture=(),
                  lazy=False):
        mean_nq = float(nq_of[lo:hi].mean())
        rate = load * sat["plain"] / mean_nq
        arrivals = np.cumsum(rng.exponential(1.0 / rate, hi - lo))
        pos = np.sort(rng.integers(lo + warm, hi, len(plan)))
        dels = [(int(pos[t]), ci, r) for t, (ci, r) in enumerate(plan)]
        srv = server(plain, bind, max_wave, lazy)
        t0 = time.perf_counter()
        lat, t_done, t_first = run.run(srv, lo, hi, arrivals=arrivals, deletions=dels,
                                       clouds=clouds, label=name, capture=capture)
        w_, r_ = srv.stats()
        srv.close()
        m = lat[warm:]
        lag, wt = run.parts[0][warm:], run.parts[1][warm:]
        t_meas = t_first + arrivals[warm] - arrivals[0]
        served = float(nq_of[lo + warm:hi].sum() / (t_done[warm:].max() - t_meas))
        out = {"p50_ms": round(float(np.percentile(m, 50)) * 1e3, 3),
               "p99_ms": round(float(np.percentile(m, 99)) * 1e3, 3),
               "mean_ms": round(float(m.mean()) * 1e3, 3),
               "mean_submit_lag_ms": round(float(lag.mean()) * 1e3, 3),
               "mean_queue_wait_ms": round(float(wt.mean()) * 1e3, 3),
               "p99_queue_wait_ms": round(float(np.percentile(wt, 99)) * 1e3, 3),
               "served_qps": round(served, 1),
               "requests_per_wave": round(r_ / max(w_, 1), 2),
               "deletion_batches": len(dels),
               "wall_s": round(time.perf_counter() - t0, 2)}
        log(f"serving: {name}: p50 {out['p50_ms']} ms, p99 {out['p99_ms']} ms, "
            f"{served / 1e6:.1f} M queries/s served, {out['requests_per_wave']} requests per wave")
        return out, dels

    # the main comparison at args.load x plain saturation, both servers from freshly packed
    # lists; the batched run keeps the rows of 200 seeded requests for the parity check
    lo, hi = nsat, nsat + nwarm + nmeas
    res = {}
    live = [np.ones(c.n, bool) for c in w.clouds]
    check = np.sort(np.random.default_rng(29).choice(np.arange(lo + nwarm, hi),
                                                     min(args.check_requests, nmeas),
                                                     replace=False))
    batched_dels = None
    for p, name in enumerate(("plain", "batched")):
        for cl in clouds:
            cl.compact()
        torch.cuda.synchronize()
        out, dels = open_loop(f"{name} open loop", lo, hi, nwarm, args.load, main_plans[p],
                              name == "plain", capture=check if name == "batched" else ())
        res[name] = out
        if name == "plain":
            for ci, r in main_plans[0]:
                live[ci][r] = False
        else:
            batched_dels = dels

    # parity: each checked request against the oracle on the live set it was answered on
    # (the deletion batches of its cloud applied before its launch, in arrival order)
    import oracle
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    from _compare import compare_rows
    per_cloud = [[] for _ in w.clouds]
    for _, ci, r in batched_dels:
        per_cloud[ci].append(r)
    thr = oracle_threads()
    ties = rows = 0
    t0 = time.perf_counter()
    for i in check:
        r = reqs[i]
        gi, gd, seen = run.captured[i]
        lv = live[r.cloud].copy()
        for b in per_cloud[r.cloud][:seen]:
            lv[b] = False
        P = w.clouds[r.cloud].by_rank
        ri, _, rD = oracle.knn_bruteforce(P, r.queries, r.k, r.m, live=lv.astype(np.uint8),
                                          threads=thr)
        ties += compare_rows(gi, gd, ri, rD, P=P, Q=r.queries, m=r.m, live=lv)
        rows += r.queries.shape[0]
    log(f"serving: parity {len(check)} requests, {rows} rows, {ties} near-tie positions "
        f"({time.perf_counter() - t0:.1f} s)")
    parity = {"requests": int(len(check)), "rows": int(rows), "near_ties": int(ties),
              "mismatches": 0, "rule": "each request on the live set of its admitted version"}
    for _, ci, r in batched_dels:
        live[ci][r] = False

    # sweep of offered loads: plain, batched (bind at admission; strict order waiting for
    # deletions; strict order filtering marked deletions) and batched without coalescing
    # (one request per wave, the same two stream slots)
    sweep = []
    lo2, hi2 = hi, hi + nsw_warm + nsw
    k = 20
    for load in loads:
        t0 = time.perf_counter()
        for cl in clouds:
            cl.compact()
        torch.cuda.synchronize()
        log(f"serving: lists re-packed for the sweep in {time.perf_counter() - t0:.1f} s")
        row = {"load": load}
        for name, plain, bind, mw, lazy in (("plain", True, True, 256, False),
                                            ("batched_bind", False, True, 256, False),
                                            ("batched_strict", False, False, 256, False),
                                            ("batched_strict_lazy", False, False, 256, True),
                                            ("batched_one_per_wave", False, True, 1, False)):
            out, dels = open_loop(f"sweep {load}x {name}", lo2, hi2, nsw_warm, load,
                                  tenth[k], plain, bind, mw, lazy=lazy)
            k += 1
            row[name] = {x: out[x] for x in ("p50_ms", "p99_ms", "served_qps",
                                             "requests_per_wave", "mean_queue_wait_ms")}
        sweep.append(row)
    return {"workload": f"serving_{len(clouds)}_clouds", "clouds": len(clouds),
            "points": int(npts), "slots": args.slots, "pool_queries": pool,
            "mean_queries_per_request": round(float(nq_of[lo:hi].mean()), 1),
            "k": list(w.k_choices),
            "saturation_qps": {"plain": round(sat["plain"], 1), "batched": round(sat["batched"], 1),
                               "requests": nsat},
            "speedup_vs_plain": round(sat["batched"] / sat["plain"], 3),
            "open_loop": {"offered": f"{args.load} x plain saturation",
                          "offered_qps": round(args.load * sat["plain"], 1),
                          "requests": nmeas, "warmup_requests": nwarm,
                          "order": "bind at admission", **res},
            "parity": parity, "sweep": sweep,
            "sweep_requests": nsw, "sweep_delete_frac_per_run": args.delete_frac / 10,
            "build_s": round(build_s, 2)}


def bench_serving(args) -> int:
    r = run_serving(args)
    b = r["saturation_qps"]["batched"]
    line = {
        "metric": METRIC, "value": b, "unit": "queries/s", "n_gpus": 1,
        "steps": args.sat_requests, "warmup": 500, "ms_per_step": None,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": r["workload"], "clouds": r["clouds"], "points": r["points"],
                   "k": r["k"], "offered_load": r["open_loop"]["offered"]},
        "extra": r,
    }
    print(json.dumps(line), flush=True)
    return 0


def bench_forms(args) -> int:
    """The batched and the serving forms, for the default run's line (run as a child
    process; with --wait-go it starts work, GPU included, when a line arrives on stdin)."""
    out = {"batched": run_batched(args), "serving": run_serving(args)}
    print(json.dumps(out), flush=True)
    return 0


def bench_dynamic(args) -> int:
    """The dynamic benchmark (insertions, queries and deletions interleaved; Sec. 5.4
    evaluation): per iteration insert 200 points, answer 2,000 queries with k=20; delete 100
    random live points every 50 iterations and insert 2,000 more every 100.  Insertions and
    deletions update the device lists (copy-on-write deltas) before the next query batch.
    Queries are drawn on the host per iteration and copied in (part of the query time)."""
    import torch
    from paper_2605_02224_amd import workloads as W
    from paper_2605_02224_amd.api import Cloud
    out = {}
    for scenario in ("surface", "volume"):
        w = W.dynamic_stream(scenario, iterations=args.dyn_iterations)
        P = w.points
        cl = Cloud.build(P[:w.n0]).upload()
        n = w.n0
        live = np.zeros(P.shape[0], bool)
        live[:n] = True
        t = collections.defaultdict(float)
        cnt = collections.defaultdict(int)
        idx = torch.empty((w.queries_per_iter, w.k), dtype=torch.int32, device="cuda")
        dist = torch.empty((w.queries_per_iter, w.k), dtype=torch.float32, device="cuda")
        torch.cuda.synchronize()
        t_all = time.perf_counter()
        for it in range(1, w.iterations + 1):
            t0 = time.perf_counter()
            cl.insert(P[n:n + w.insert_per_iter])
            live[n:n + w.insert_per_iter] = True
            n += w.insert_per_iter
            t1 = time.perf_counter()
            t["insert"] += t1 - t0
            cnt["insert"] += w.insert_per_iter
            q = W.uniform_in_box(w.rng, w.queries_per_iter, w.qlo, w.qhi)
            qd = torch.from_numpy(q).cuda(non_blocking=False)
            cl.knn(qd, w.k, out=(idx, dist))
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            t["query"] += t2 - t1
            cnt["query"] += w.queries_per_iter
            if it % w.delete_every == 0:
                dead = w.rng.choice(np.flatnonzero(live), w.delete_count, replace=False)
                cl.delete(dead)
                live[dead] = False
                t3 = time.perf_counter()
                t["delete"] += t3 - t2
                cnt["delete"] += w.delete_count
                t2 = t3
            if it % w.batch_every == 0:
                cl.insert(P[n:n + w.batch_count])
                live[n:n + w.batch_count] = True
                n += w.batch_count
                t["insert"] += time.perf_counter() - t2
                cnt["insert"] += w.batch_count
        total = time.perf_counter() - t_all
        log(f"{scenario}: {w.iterations} iterations in {total:.2f} s; final n={n}, "
            f"live={cl.live_count}")
        out[scenario] = {
            "total_s": round(total, 3),
            "insert_us_per_point": round(1e6 * t["insert"] / max(cnt["insert"], 1), 2),
            "query_ms_per_iteration": round(1e3 * t["query"] / w.iterations, 4),
            "queries_per_s": round(cnt["query"] / t["query"], 1),
            "delete_us_per_point": round(1e6 * t["delete"] / max(cnt["delete"], 1), 2),
            "final_points": int(n), "final_live": int(cl.live_count),
        }
    line = {
        "metric": "dynamic benchmark: total time of the interleaved insert/query/delete run",
        "value": out["surface"]["total_s"], "unit": "s", "n_gpus": 1,
        "steps": args.dyn_iterations, "warmup": 0,
        "ms_per_step": round(1e3 * out["surface"]["total_s"] / args.dyn_iterations, 3),
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "dynamic_5k_plus_200_per_iteration_k20",
                   "iterations": args.dyn_iterations, "n0": 5000, "insert_per_iteration": 200,
                   "queries_per_iteration": 2000, "k": 20, "delete": "100 every 50",
                   "batch_insert": "2000 every 100"},
        "extra": out,
    }
    print(json.dumps(line), flush=True)
    return 0


def bench_plane(args) -> int:
    """k-NN with a plane fit per row (the scan convergence statistic): the headline cloud
    (torus, 1M points), 1M probes near the surface (torus samples jittered by 1e-2), k=20,
    m=n; against the same queries without the fit."""
    import torch
    from paper_2605_02224_amd import workloads as W
    from paper_2605_02224_amd.api import Cloud
    w = W.torus_paper_scale(n=args.n, nq=args.nq, k=20)
    cl = Cloud.build(w.cloud.by_rank).upload()
    q = torch.from_numpy(w.queries_b).cuda()
    nq, k = q.shape[0], 20
    res = {}
    for name, fn in (("knn", lambda: cl.knn(q, k)), ("knn_plane", lambda: cl.knn_plane(q, k))):
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            fn()
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / args.steps
        res[name] = (nq / dt, dt)
        log(f"{name}: {nq / dt / 1e6:.1f} M queries/s, {dt * 1e3:.3f} ms per batch")
    line = {
        "metric": "k-NN + local plane fit: probes/s",
        "value": round(res["knn_plane"][0], 1), "unit": "queries/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(res["knn_plane"][1] * 1e3, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "torus_1M_surface_probes_k20_plane_fit", "n": args.n,
                   "nq": nq, "k": k},
        "extra": {"knn_only_qps": round(res["knn"][0], 1),
                  "fit_overhead": round(res["knn_plane"][1] / res["knn"][1] - 1, 4)},
    }
    print(json.dumps(line), flush=True)
    return 0


def _forms_argv(args):
    """Command line of the child process that measures the batched and serving forms."""
    return [sys.executable, os.path.abspath(__file__), "--workload", "forms", "--wait-go",
            "--steps", str(max(3, args.steps // 2)), "--warmup", str(max(1, args.warmup)),
            "--clouds", str(args.clouds), "--tile", str(args.tile),
            "--serving-clouds", str(args.serving_clouds),
            "--serving-n-hi", str(args.serving_n_hi), "--requests", str(args.requests),
            "--warm-requests", str(args.warm_requests), "--sat-requests", str(args.sat_requests),
            "--load", str(args.load), "--slots", str(args.slots),
            "--delete-frac", str(args.delete_frac), "--check-requests", str(args.check_requests),
            "--sweep-loads", args.sweep_loads, "--sweep-requests", str(args.sweep_requests)] + \
        (["--no-autotune"] if args.no_autotune else [])


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="torus",
                    choices=["torus", "batched", "serving", "forms", "dynamic", "plane"])
    ap.add_argument("--dyn-iterations", type=int, default=2000, help="dynamic: iterations")
    ap.add_argument("--requests", type=int, default=20000, help="serving: measured requests")
    ap.add_argument("--warm-requests", type=int, default=1000)
    ap.add_argument("--sat-requests", type=int, default=5000)
    ap.add_argument("--load", type=float, default=0.7, help="serving: x plain saturation")
    ap.add_argument("--slots", type=int, default=2, help="serving: stream slots")
    ap.add_argument("--serving-clouds", type=int, default=64)
    ap.add_argument("--serving-n-hi", type=int, default=2_000_000)
    ap.add_argument("--delete-frac", type=float, default=0.01,
                    help="serving: fraction of each cloud deleted during a main run")
    ap.add_argument("--check-requests", type=int, default=200,
                    help="serving: requests checked against the oracle")
    ap.add_argument("--sweep-loads", default="0.25,0.5,0.9,1.2",
                    help="serving: offered loads of the sweep (x plain saturation), or ''")
    ap.add_argument("--sweep-requests", type=int, default=2000)
    ap.add_argument("--clouds", type=int, default=256, help="batched: clouds")
    ap.add_argument("--tile", type=int, default=16)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=1_000_000)
    ap.add_argument("--nq", type=int, default=1_000_000)
    ap.add_argument("--k", type=int, default=16)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="skip the context measurements")
    ap.add_argument("--layout-probe", action="store_true",
                    help="time the other list layouts beside the records even with --no-extras")
    ap.add_argument("--no-forms", action="store_true",
                    help="skip the batched and serving forms (child process)")
    ap.add_argument("--no-autotune", action="store_true", help="use the built-in configuration")
    ap.add_argument("--no-host-build", action="store_true",
                    help="skip the host construction the device-built lists are compared with")
    ap.add_argument("--wait-go", action="store_true", help=argparse.SUPPRESS)
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run one plain 1 GiB device copy (to scale HBM byte counters)")
    ap.add_argument("--ingest-counters", nargs=3, metavar=("FETCH_DIR", "WRITE_DIR", "OUT"),
                    help="write the HBM traffic reading from two rocprofv3 --pmc runs")
    ap.add_argument("--trace-summary", metavar="TRACE_DIR",
                    help="durations of the headline kernel in a rocprofv3 kernel trace")
    args = ap.parse_args()
    if args.ingest_counters:
        print(json.dumps(ingest_counters(*args.ingest_counters, last=args.steps)))
        return 0
    if args.trace_summary:
        print(json.dumps(trace_summary(args.trace_summary, last=args.steps), indent=1))
        return 0
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU: the query path has no "
                                   "multi-GPU form, so --gpus must be 1"}))
        return 2

    # the forms run in a child process started before this process touches the GPU; it
    # waits for a line on its stdin, sent once the headline measurement is done
    if args.workload == "forms" and args.wait_go:
        sys.stdin.readline()          # the parent is done with the GPU: start now
    child = None
    if args.workload == "torus" and not args.no_forms:
        import subprocess
        child = subprocess.Popen(_forms_argv(args), stdin=subprocess.PIPE,
                                 stdout=subprocess.PIPE, text=True)
    try:
        return _main(args, child)
    finally:
        if child is not None and child.poll() is None:
            child.kill()
            child.wait()


def _main(args, child) -> int:
    import torch
    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        return 2
    if args.workload == "batched":
        return bench_batched(args)
    if args.workload == "dynamic":
        return bench_dynamic(args)
    if args.workload == "plane":
        return bench_plane(args)
    if args.workload == "serving":
        return bench_serving(args)
    if args.workload == "forms":
        return bench_forms(args)
    from paper_2605_02224_amd import workloads as W
    from paper_2605_02224_amd import _lib
    from paper_2605_02224_amd.api import Cloud

    t0 = time.perf_counter()
    w = W.torus_paper_scale(n=args.n, nq=args.nq, k=args.k)
    P = w.cloud.by_rank
    log(f"workload generated in {time.perf_counter() - t0:.1f} s")
    # the lists, built on the GPU (timed), and by the host construction for comparison
    from paper_2605_02224_amd import api as A
    Cloud.build(P[:1000], device=True)   # first use of the device path (code objects load)
    t0 = time.perf_counter()
    cl = Cloud.build(P, device=True)
    build_dev_s = time.perf_counter() - t0
    build_stats = A.build_device_stats()
    build_s, lists_equal = None, None
    if not args.no_host_build:
        t0 = time.perf_counter()
        cl_host = Cloud.build(P)
        build_s = time.perf_counter() - t0
        ho, he = cl_host.successors()
        do, de = cl.successors()
        lists_equal = bool(np.array_equal(ho, do) and np.array_equal(he, de))
        del cl_host, ho, he, do, de
        if not lists_equal:
            raise RuntimeError("device-built lists differ from the host construction's")
    log(f"lists built on the GPU in {build_dev_s:.2f} s ({build_stats}), on the host in "
        f"{build_s} s; equal: {lists_equal}")
    cl.upload()
    q = torch.from_numpy(w.queries).cuda()
    qb = torch.from_numpy(w.queries_b).cuda()
    nq = q.shape[0]
    k = args.k
    idx = torch.empty((nq, k), dtype=torch.int32, device="cuda")
    dist = torch.empty((nq, k), dtype=torch.float32, device="cuda")
    torch.cuda.synchronize()

    # algorithmic bytes per query: 16 B per list entry examined, 8 B per list opened,
    # 12 B query, 8 B per output neighbour (rank + distance)
    ce, cn, ci = cl.knn_counts(q, k, inserts=True)
    torch.cuda.synchronize()
    E = ce.double().mean().item()
    L = cn.double().mean().item()
    INS = ci.double().mean().item()
    bytes_per_q = 16.0 * E + 8.0 * L + 12.0 + 8.0 * k
    log(f"per query: {E:.1f} entries, {L:.2f} lists, {INS:.1f} inserts -> "
        f"{bytes_per_q:.0f} algorithmic bytes")

    # autotuner (untimed): picks the kernel configuration for this size and k class
    tuned = None
    if not args.no_autotune:
        from paper_2605_02224_amd import api as A
        t0 = time.perf_counter()
        best, tried = A.autotune(cl, q, k)
        tuned = dict(best, seconds=round(time.perf_counter() - t0, 3))
        log(f"autotuner: {best} of {len(tried)} candidates")
    for _ in range(args.warmup):
        cl.knn(q, k, out=(idx, dist))
    torch.cuda.synchronize()
    lib = _lib.lib()
    lib.mknn_timing_enable(1)
    import ctypes
    tot = ctypes.c_double()
    cnt = ctypes.c_int64()
    lib.mknn_timing_read(ctypes.byref(tot), ctypes.byref(cnt))   # reset
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        cl.knn(q, k, out=(idx, dist))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    _lib.check(lib.mknn_timing_read(ctypes.byref(tot), ctypes.byref(cnt)))
    lib.mknn_timing_enable(0)
    ms_step = 1e3 * wall / args.steps
    qps = nq * args.steps / wall
    kern_ms = tot.value / max(cnt.value, 1)
    achieved = bytes_per_q * nq / (kern_ms * 1e-3) / 1e9
    log(f"{qps / 1e6:.1f} M queries/s, {ms_step:.3f} ms/step, query kernel {kern_ms:.3f} ms")
    gpu_idx = idx.cpu().numpy()
    gpu_dist = dist.cpu().numpy()

    # context numbers (not the headline): k=1 and the on-surface query set
    traffic = measured_traffic(k)
    extras = {"build_s": None if build_s is None else round(build_s, 2),
              "build_device_s": round(build_dev_s, 3),
              "build_device": {k: (round(v, 1) if isinstance(v, float) else v)
                               for k, v in build_stats.items()},
              "build_lists_equal": lists_equal, "device_bytes": cl.device_bytes,
              "entries_per_query": round(E, 2), "lists_per_query": round(L, 3),
              "inserts_per_query": round(INS, 2), "algorithmic_bytes_per_query": round(bytes_per_q, 1),
              "kernel": f"mknn::{HEADLINE_KERNEL} (k={k})" if k == 16 else None,
              "kernel_ms": round(kern_ms, 4), "autotuned": tuned,
              "roofline_frac_step_basis": round(qps * bytes_per_q / (HBM_PEAK_GBS * 1e9), 4),
              "hbm_measured_GBps": (round(traffic / (kern_ms * 1e-3) / 1e9, 1)
                                    if traffic else None)}
    extra_runs = () if args.no_extras else (("volume_k1", q, 1), ("surface_k16", qb, 16),
                                            ("surface_k1", qb, 1))
    for name, qq, kk in extra_runs:
        i2 = torch.empty((nq, kk), dtype=torch.int32, device="cuda")
        d2 = torch.empty((nq, kk), dtype=torch.float32, device="cuda")
        for _ in range(2):
            cl.knn(qq, kk, out=(i2, d2))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        reps = max(3, args.steps // 4)
        for _ in range(reps):
            cl.knn(qq, kk, out=(i2, d2))
        torch.cuda.synchronize()
        extras[name + "_qps"] = round(nq * reps / (time.perf_counter() - t0), 1)
    if not args.no_extras or args.layout_probe:
        extras["layout_probe"] = layout_probe(cl, q, idx, dist, kern_ms, args.steps, k)
        log(f"layout probe: {extras['layout_probe']}")
    if not args.no_extras:
        probe = memory_probes()
        probe["frac_of_stream_read"] = round(achieved / probe["stream_read_GBps"], 4)
        extras["memory_probe"] = probe
        log(f"memory probes: {probe}")
    log(f"extras: {extras}")

    if args.copy_probe:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")   # 1 GiB
        dst = torch.empty_like(src)
        torch.mul(src, 2.0, out=dst)          # one elementwise pass: reads and writes 1 GiB
        torch.cuda.synchronize()
        del src, dst
        log("copy probe: elementwise kernel reading 1 GiB and writing 1 GiB")

    cpu = None
    if not args.no_cpu_baseline:
        cpu, parity = cpu_baseline(P, w.queries, k, args.cpu_seconds, gpu_idx, gpu_dist)
        extras["parity"] = parity
        log(f"cpu baseline: {cpu}; parity: {parity}")

    if child is not None:
        log("starting the batched and serving forms (child process)")
        out, _ = child.communicate("go\n")
        if child.returncode != 0:
            raise RuntimeError(f"the batched/serving child process failed ({child.returncode})")
        forms = json.loads(out.strip().splitlines()[-1])
        extras["batched"] = forms["batched"]
        extras["serving"] = forms["serving"]

    line = {
        "metric": METRIC,
        "value": round(qps, 1),
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "torus_1M_volume_queries_k16", "n": args.n, "nq": nq, "k": k,
                   "m": args.n, "form": "plain (one launch per batch)",
                   "queries": "uniform in bbox x1.1", "order": "seeded random"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic},
        "cpu_baseline": cpu,
        "extra": extras,
    }
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
