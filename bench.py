#!/usr/bin/env python3
"""Benchmark of the Manifold k-NN query path on one MI355X.

A step is one pass of the whole query path over one batch: the query batch preparation
(Morton bucketing), the 1-NN descent (Alg. 1) and the k-expansion (Alg. 2) with the prefix
bound, writing indices and distances -- for the headline workload: 1,000,000 points on a
torus (R=1, r=0.3, normal noise 1e-3, random insertion order), 1,000,000 volume queries
uniform in the bounding box expanded by 10%, k=16, m=n.  Inputs are resident in HBM
before timing starts; the host-side list construction is reported but not timed.

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


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def csrc_digest() -> str:
    """Hash of the sources the kernels are compiled from (the HIP translation units and
    every header), to tell whether stored counter readings still apply.  Host-only C++
    (construction, deletion, insertion) does not enter."""
    import glob
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2605_02224_amd", "csrc")
    files = glob.glob(os.path.join(csrc, "*.hip")) + glob.glob(os.path.join(csrc, "*.h"))
    for f in sorted(files):
        h.update(os.path.basename(f).encode())
        h.update(open(f, "rb").read())
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
    return 1024.0 * (rec["fetch_kib_per_dispatch"] * rec["fetch_scale"] +
                     rec["write_kib_per_dispatch"] * rec["write_scale"])


def cpu_baseline(P, Q, k, target_s: float):
    """Time the FP64 brute-force oracle on a bounded sample of the same queries."""
    import oracle
    oracle.build(force=False)
    threads = oracle.max_threads()
    oracle.knn_bruteforce(P, Q[:16], k)           # load the library, start the threads
    n0 = min(64, Q.shape[0])
    while True:
        t = time.perf_counter()
        oracle.knn_bruteforce(P, Q[:n0], k)
        dt = max(time.perf_counter() - t, 1e-6)
        if dt >= 0.5 or n0 >= Q.shape[0]:
            break
        n0 = min(Q.shape[0], n0 * 4)
    ns = int(min(Q.shape[0], max(n0, n0 * target_s / dt)))
    t = time.perf_counter()
    oracle.knn_bruteforce(P, Q[:ns], k)
    dt = time.perf_counter() - t
    return {"value": ns / dt, "unit": "queries/s", "cores": threads, "kind": "oracle",
            "sample": f"first {ns} of the {Q.shape[0]} timed queries, brute force over all "
                      f"{P.shape[0]} points, FP64, {dt:.1f} s wall"}


def build_clouds(clouds, threads: int = 16):
    """Build and upload many clouds; host construction runs on a thread pool (the C call
    releases the GIL)."""
    import concurrent.futures as cf
    from paper_2605_02224_amd.api import Cloud
    with cf.ThreadPoolExecutor(max_workers=threads) as ex:
        built = list(ex.map(lambda c: Cloud.build(c.by_rank), clouds))
    for c in built:
        c.upload()
    return built


def bench_batched(args) -> int:
    """Many clouds (sizes log-uniform in [1e3, 2e5], sphere/torus/ellipsoid, 4 n_c queries
    each, k=10): one flat launch per class and batch versus one plain launch per cloud."""
    import torch
    from paper_2605_02224_amd import workloads as W
    from paper_2605_02224_amd import api as A
    t0 = time.perf_counter()
    w = W.many_clouds(num=args.clouds)
    log(f"{len(w.clouds)} clouds, {sum(c.n for c in w.clouds)} points generated in "
        f"{time.perf_counter() - t0:.1f} s")
    t0 = time.perf_counter()
    clouds = build_clouds(w.clouds)
    build_s = time.perf_counter() - t0
    log(f"built and uploaded in {build_s:.1f} s")
    qs = [torch.from_numpy(q).cuda() for q in w.queries]
    nq = sum(q.shape[0] for q in qs)
    items = A.alloc_outputs([(c, q, w.k, None) for c, q in zip(clouds, qs)])
    plan = A.BatchPlan(len(items), nq, tile_queries=args.tile, sort=True, graph=True)
    tile = args.tile
    if not args.no_autotune:
        tile = plan.tune(items)   # untimed: picks the tile length for this batch
        log(f"autotuner: tile length {tile}")
    torch.cuda.synchronize()

    def run_batched():
        plan.run(items)

    def run_plain():
        for cl, q, k, m, idx, dist in items:
            cl.knn(q, k, out=(idx, dist))

    res = {}
    for name, fn in (("plain", run_plain), ("batched", run_batched)):
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            fn()
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / args.steps
        res[name] = (nq / dt, dt)
        log(f"{name}: {nq / dt / 1e6:.1f} M queries/s, {dt * 1e3:.2f} ms per batch")
    line = {
        "metric": "k-NN queries/sec (k=16, 1M-pt surface) + p50/p99 latency, batched vs plain",
        "value": round(res["batched"][0], 1), "unit": "queries/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(res["batched"][1] * 1e3, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"batched_{len(items)}_clouds_k{w.k}", "clouds": len(items),
                   "points": int(sum(c.n for c in w.clouds)), "queries": int(nq), "k": w.k,
                   "form": "one flat launch per class (hipGraph replay) per batch",
                   "tile_queries": tile},
        "extra": {"plain_qps": round(res["plain"][0], 1),
                  "plain_ms": round(res["plain"][1] * 1e3, 3),
                  "speedup_vs_plain": round(res["batched"][0] / res["plain"][0], 3),
                  "build_s": round(build_s, 2)},
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

    def run(self, srv, lo, hi, arrivals=None, deletions=(), clouds=None, label=""):
        """Requests lo..hi-1; arrivals: offsets in seconds from the start (None = as fast as
        the ring allows); deletions: (position, cloud, ranks) submitted just before the
        request at that position.  Returns per-request latencies and the makespan."""
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


def bench_serving(args) -> int:
    """Serving: 64 resident clouds (sizes log-uniform in [1e4, 2e6], about 24M points),
    requests of 1..65536 queries (log-uniform), k in {4, 16, 64}, prefix m uniform in
    [n/10, n]; open-loop Poisson arrivals at 0.7x the plain server's saturation rate; 1% of
    the points deleted in batches of <= 1000 between requests.  The batched server
    (continuous batching on stream slots) against the plain one (one launch per request)."""
    import torch
    from paper_2605_02224_amd import workloads as W
    from paper_2605_02224_amd import api as A
    sys.setswitchinterval(2e-4)   # the submitter and the collector hand the GIL over quickly
    t0 = time.perf_counter()
    w = W.serving_clouds(num=args.clouds, n_hi=args.serving_n_hi)
    npts = sum(c.n for c in w.clouds)
    log(f"{len(w.clouds)} clouds, {npts} points generated in {time.perf_counter() - t0:.1f} s")
    t0 = time.perf_counter()
    clouds = build_clouds(w.clouds)
    build_s = time.perf_counter() - t0
    log(f"built and uploaded in {build_s:.1f} s")
    nwarm, nmeas, nsat = args.warm_requests, args.requests, args.sat_requests
    total = nsat + nwarm + nmeas
    t0 = time.perf_counter()
    reqs = [w.request() for _ in range(total)]
    log(f"{total} requests generated in {time.perf_counter() - t0:.1f} s")
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
    log(f"{int(qoff[-1])} queries resident, output ring of {cap} entries; host cpus "
        f"{len(os.sched_getaffinity(0))}")
    nq_of = np.diff(qoff)
    pool = 1 << 22
    kw = dict(pool_queries=pool, nstreams=args.slots, max_wave_requests=256,
              bind_at_admission=True)

    def server(plain):
        return A.Server(plain=plain, **kw)

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
        log(f"{name} saturation: {sat[name] / 1e6:.1f} M queries/s "
            f"({nsat / span:.0f} requests/s, {r_ / max(w_, 1):.1f} requests per wave)")
    # open loop at 0.7x the plain saturation rate, with deletions
    lo, hi = nsat, total
    mean_nq = float(nq_of[lo:hi].mean())
    rate = args.load * sat["plain"] / mean_nq
    rng = np.random.default_rng(11)
    arrivals = np.cumsum(rng.exponential(1.0 / rate, hi - lo))
    parts = w.deletion_plan(frac=args.delete_frac, batch=1000, parts=2)
    res = {}
    for p, name in enumerate(("plain", "batched")):
        for cl in clouds:          # both runs start from freshly packed lists
            cl.compact()
        torch.cuda.synchronize()
        pos = np.sort(rng.integers(lo + nwarm, hi, len(parts[p])))
        dels = [(int(pos[t]), ci, r) for t, (ci, r) in enumerate(parts[p])]
        srv = server(name == "plain")
        t0 = time.perf_counter()
        lat, t_done, t_first = run.run(srv, lo, hi, arrivals=arrivals, deletions=dels,
                                       clouds=clouds, label=f"{name} open loop")
        w_, r_ = srv.stats()
        srv.close()
        m = lat[nwarm:]
        lag, wt = run.parts[0][nwarm:], run.parts[1][nwarm:]
        t_meas = t_first + arrivals[nwarm] - arrivals[0]
        served = float(nq_of[lo + nwarm:hi].sum() / (t_done[nwarm:].max() - t_meas))
        res[name] = {"p50_ms": round(float(np.percentile(m, 50)) * 1e3, 3),
                     "p99_ms": round(float(np.percentile(m, 99)) * 1e3, 3),
                     "mean_ms": round(float(m.mean()) * 1e3, 3),
                     "mean_submit_lag_ms": round(float(lag.mean()) * 1e3, 3),
                     "mean_queue_wait_ms": round(float(wt.mean()) * 1e3, 3),
                     "p99_queue_wait_ms": round(float(np.percentile(wt, 99)) * 1e3, 3),
                     "served_qps": round(served, 1),
                     "requests_per_wave": round(r_ / max(w_, 1), 2),
                     "deletion_batches": len(dels),
                     "wall_s": round(time.perf_counter() - t0, 2)}
        log(f"{name} open loop: p50 {res[name]['p50_ms']} ms, p99 {res[name]['p99_ms']} ms, "
            f"{served / 1e6:.1f} M queries/s served; mean submit lag "
            f"{res[name]['mean_submit_lag_ms']} ms, mean queue wait "
            f"{res[name]['mean_queue_wait_ms']} ms")
    line = {
        "metric": "k-NN queries/sec (k=16, 1M-pt surface) + p50/p99 latency, batched vs plain",
        "value": round(sat["batched"], 1), "unit": "queries/s", "n_gpus": 1,
        "steps": nsat, "warmup": 500,
        "ms_per_step": round(1e3 * nq_of[:nsat].sum() / sat["batched"] / nsat, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"serving_{len(clouds)}_clouds", "clouds": len(clouds),
                   "points": int(npts), "requests_saturation": nsat,
                   "requests_open_loop": nmeas, "warmup_requests": nwarm,
                   "mean_queries_per_request": round(mean_nq, 1), "k": [4, 16, 64],
                   "offered_load": f"{args.load} x plain saturation",
                   "offered_qps": round(args.load * sat["plain"], 1),
                   "slots": args.slots, "pool_queries": pool,
                   "order": "bind at admission"},
        "extra": {"plain_saturation_qps": round(sat["plain"], 1),
                  "speedup_vs_plain": round(sat["batched"] / sat["plain"], 3),
                  "open_loop": res, "build_s": round(build_s, 2)},
    }
    print(json.dumps(line), flush=True)
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


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="torus",
                    choices=["torus", "batched", "serving", "dynamic", "plane"])
    ap.add_argument("--dyn-iterations", type=int, default=2000, help="dynamic: iterations")
    ap.add_argument("--requests", type=int, default=20000, help="serving: measured requests")
    ap.add_argument("--warm-requests", type=int, default=1000)
    ap.add_argument("--sat-requests", type=int, default=5000)
    ap.add_argument("--load", type=float, default=0.7, help="serving: x plain saturation")
    ap.add_argument("--slots", type=int, default=2, help="serving: stream slots")
    ap.add_argument("--serving-n-hi", type=int, default=2_000_000)
    ap.add_argument("--delete-frac", type=float, default=0.01,
                    help="serving: fraction of each cloud deleted during a run")
    ap.add_argument("--clouds", type=int, default=256)
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
    ap.add_argument("--no-autotune", action="store_true", help="use the built-in configuration")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run one plain 1 GiB device copy (to scale HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU only; --gpus must be 1"}))
        return 2

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
        if args.clouds == 256:
            args.clouds = 64
        return bench_serving(args)
    from paper_2605_02224_amd import workloads as W
    from paper_2605_02224_amd import _lib
    from paper_2605_02224_amd.api import Cloud

    t0 = time.perf_counter()
    w = W.torus_paper_scale(n=args.n, nq=args.nq, k=args.k)
    P = w.cloud.by_rank
    log(f"workload generated in {time.perf_counter() - t0:.1f} s")
    t0 = time.perf_counter()
    cl = Cloud.build(P)
    build_s = time.perf_counter() - t0
    log(f"lists built in {build_s:.1f} s")
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

    # context numbers (not the headline): k=1 and the on-surface query set
    extras = {"build_s": round(build_s, 2), "device_bytes": cl.device_bytes,
              "entries_per_query": round(E, 2), "lists_per_query": round(L, 3),
              "inserts_per_query": round(INS, 2),
              "kernel_ms": round(kern_ms, 4), "autotuned": tuned}
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
        cpu = cpu_baseline(P, w.queries, k, args.cpu_seconds)
        log(f"cpu baseline: {cpu}")

    line = {
        "metric": "k-NN queries/sec (k=16, 1M-pt surface) + p50/p99 latency, batched vs plain",
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
                     "traffic": measured_traffic(k)},
        "cpu_baseline": cpu,
        "extra": extras,
    }
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
