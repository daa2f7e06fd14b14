#!/usr/bin/env python3
"""Benchmark: exact k <= 4 graphlet counts on one MI355X.

Default workload: R-MAT scale 22 (edge factor 16, a,b,c,d = .57,.19,.19,.05,
64.2M undirected edges after symmetrising and deduplicating), full 17-class
counts, CSR resident in HBM before the timed region.  One step = one
graphlet_count call (prepass, Steps 1-4, result on the host).

Prints one JSON line (the last line of stdout).  The default line also
carries the other two parts of the metric, compact: "batched" (the 8192-graph
batch, as --workload batch) and "serve" (the Poisson trace, as --workload
serve); --no-extras leaves them out.  Other workloads:
  --workload er | cl       the other single-graph configurations
  --workload batch         8192 small graphs in one batched call, against one
                           plain call per graph
  --workload serve         Poisson request stream through the serving loop,
                           against plain per-request launches
  --workload update        single-edge deletions and insertions on R-MAT
                           scale 22 by localized update, against a recount
  --workload vertex        per-vertex counts (17 per vertex) of R-MAT scale 22
  --workload batch_vertex  per-vertex counts of every vertex of the 8192-graph
                           batch in one call, against one call per graph
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, GB/s
# 32-bit integer vector lane operations per second: 256 compute units x 4
# SIMDs x 16 lanes per clock x 2.4 GHz (the fp32 vector rate of 157.3 TFLOP/s
# is twice this for an FMA's two operations and twice again for packed fp32;
# integer AND and popcount are one operation on one lane each)
ALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def host_cpu() -> dict:
    """This host's CPU model and logical core count (the oracle runs on one)."""
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"cpu_model": model, "nproc": os.cpu_count()}


def stored_oracle(name: str):
    """The stored oracle entry of a workload (tests/golden/configs.json)."""
    path = os.path.join(ROOT, "tests", "golden", "configs.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        return json.load(f).get(name)


def per_edge_oracle_rate(g, seconds: float, seed: int = 0):
    """The oracle's per-edge route (|Tri_e|, 4-cliques, induced 4-cycles of
    one edge by their definitions) on uniformly sampled edges of the graph,
    run for about `seconds` on one host core: (edges/s, edges, seconds)."""
    import numpy as np

    import oracle

    eu, ev = oracle.edges(g)
    rng = np.random.default_rng(seed)
    order = rng.permutation(len(eu))
    done, t0 = 0, time.perf_counter()
    chunk = 16
    while time.perf_counter() - t0 < seconds and done < len(order):
        idx = order[done:done + chunk]
        oracle.per_edge(g, eu[idx], ev[idx])
        done += len(idx)
        chunk = min(chunk * 2, 4096)
    dt = time.perf_counter() - t0
    return done / dt, done, dt


def identity_route_sample(name: str):
    """The oracle's global-count route (Chiba-Nishizeki listing, degree-ordered
    wedges and subset-sum identities) on a bounded stand-in of the workload,
    timed on this host, one core: (edges/s, description).  R-MAT: the same
    generator and parameters at scale 17 (1.9M edges, about 15 s); Chung-Lu:
    a fifth of the nodes and balls; Erdos-Renyi: the whole graph."""
    import graphgen
    import graphgen.configs as C
    import oracle

    if name == "rmat":
        p = C.RMAT
        scale = 17
        g = graphgen.rmat(scale, p["edge_factor"], p["a"], p["b"], p["c"], p["seed"])
        what = (f"R-MAT scale {scale} (n={g.n}, m={g.m}), the same generator parameters "
                f"(edge factor {p['edge_factor']}, a,b,c = {p['a']},{p['b']},{p['c']}); "
                "the route's edge rate falls as the graph grows")
    elif name == "cl":
        p = C.CL
        n, balls = p["n"] // 5, p["balls"] // 5
        g = graphgen.chung_lu(n, p["beta"], p["i0"], balls, p["seed"])
        what = (f"Chung-Lu with a fifth of the nodes and balls (n={g.n}, m={g.m}), exponent "
                f"{p['beta']}, offset {p['i0']}")
    else:
        g = C.er()
        what = f"the whole graph (n={g.n}, m={g.m})"
    t0 = time.perf_counter()
    oracle.identity_route(g)
    dt = time.perf_counter() - t0
    return g.m / dt, f"{what}, {dt:.1f} s"


def cpu_baseline(g, name: str, seconds: float):
    """The oracle beside the GPU for a global-count workload, on this host's
    cores (one used).

    value: the identity route (the oracle's global-count route) timed live on
    a bounded stand-in of the workload (identity_route_sample).  Beside it:
    the same route's stored time on the whole graph (taken when the stored
    counts were written, on the host named there), and the per-edge route
    (the literal per-edge definitions) on sampled edges of the same graph for
    `seconds`."""
    rate_s, what = identity_route_sample(name)
    rate, done, dt = per_edge_oracle_rate(g, seconds)
    res = {"value": rate_s, "unit": "edges/s", "cores": 1, "kind": "oracle",
           "route": "oracle.identity_route (global counts)", "sample": what,
           "host": host_cpu(),
           "per_edge_route": {"value": rate, "unit": "edges/s", "cores": 1,
                              "route": "oracle.per_edge",
                              "sample": f"{done} uniformly sampled edges of the same graph, "
                                        f"{dt:.1f} s"}}
    st = stored_oracle(name)
    if st is not None and st.get("sha256") == g.sha256() and st.get("oracle_seconds"):
        res["whole_graph_stored"] = {
            "value": g.m / st["oracle_seconds"], "unit": "edges/s", "cores": 1,
            "seconds": st["oracle_seconds"],
            "host": st.get("host", {"cpu_model": "the build container (8-core Xeon), "
                                                 "model not stored"})}
    return res


TRAFFIC_PROFILES = {"rmat22": "k_c4_heavy_bal_rmat22_traffic.md",
                    "cl": "k_c4_heavy_bal_chung_lu_per_edge_traffic.md"}
TRAFFIC_SOURCES = ["paper_1506_04322_amd/csrc/cycles.hip", "paper_1506_04322_amd/csrc/kernels.h",
                   "paper_1506_04322_amd/csrc/common.h"]


def measured_traffic(kernel: str, workload: str, field: str = "traffic_bytes_per_launch"):
    """HBM bytes per launch of `kernel` (or another recorded field, such as
    its L2 hit rate) from the committed rocprofv3 counters, or None when they
    were taken on other sources or another workload."""
    path = os.path.join(ROOT, "profiles", TRAFFIC_PROFILES.get(workload, "-"))
    if not os.path.exists(path):
        return None
    fields = {}
    for line in open(path):
        if ":" in line and not line.startswith(("|", "#", "`")):
            k, v = line.split(":", 1)
            fields[k.strip()] = v.strip()
    if fields.get("kernel") != kernel:
        return None
    h = hashlib.sha256()
    for rel in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    if h.hexdigest() != fields.get("source_sha256") or field not in fields:
        return None
    return float(fields[field])


def roofline_from_timing(t: dict, per_edge: bool = False):
    """The dominant kernel, the heavy 4-cycle items (one launch, alone in its
    phase; k_c4_heavy_bal, its per-edge instantiation with per-edge
    outputs): its algorithmic bytes (4 B per wedge it aggregates) over its
    device time from HIP events on the library's stream."""
    ms, nbytes = t["cyc_heavy_ms"], 4 * t["wedges_heavy"]
    achieved = nbytes / (ms / 1e3) / 1e9 if ms > 0 else 0.0
    return "cyc_heavy", {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                         "traffic": None,
                         "kernel": "k_c4_heavy_bal<true>" if per_edge else "k_c4_heavy_bal",
                         "phase_ms": round(ms, 3),
                         "bytes_per_launch": nbytes,
                         "work_unit": "wedges of the heavy work items x 4 B"}


def run_single(args, torch, gl):
    import graphgen.configs as C

    builders = {"rmat22": (C.rmat22, C.RMAT), "er": (C.er, C.ER), "cl": (C.cl, C.CL)}
    build, params = builders[args.workload]
    # the Chung-Lu configuration also writes the per-edge |Tri_e|, 4-clique
    # and induced 4-cycle arrays
    per_edge = args.workload == "cl"
    t0 = time.time()
    g = build()
    log(f"[bench] generated {args.workload}: n={g.n} m={g.m} in {time.time() - t0:.1f}s")
    dev = torch.device("cuda:0")
    torch.cuda.synchronize()
    t_up = time.perf_counter()
    rp = torch.from_numpy(g.row_ptr).to(dev)
    col = torch.from_numpy(g.col).to(dev)
    torch.cuda.synchronize()
    h2d_ms = (time.perf_counter() - t_up) * 1e3  # pageable host CSR -> HBM, not in value
    ws_bytes = gl.graphlet_workspace_size(rp, col, g.n, per_edge=per_edge)
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device=dev)
    pe = torch.empty((3, max(g.m, 1)), dtype=torch.int64, device=dev) if per_edge else None
    log(f"[bench] workspace {ws_bytes / 2**30:.2f} GiB")

    def call():
        if per_edge:
            return gl.graphlet_count(rp, col, g.n, per_edge=True, workspace=ws,
                                     per_edge_out=pe)[0]
        return gl.graphlet_count(rp, col, g.n, workspace=ws)

    gl.graphlet_timing_enable(True)
    counts = None
    for i in range(args.warmup):
        counts = call()
        log(f"[bench] warmup {i} done")
    torch.cuda.synchronize()
    phase_sum = {}
    step_ms = []
    t0 = time.perf_counter()
    for i in range(args.steps):
        ts = time.perf_counter()
        c = call()  # returns with the counts on the host
        step_ms.append((time.perf_counter() - ts) * 1e3)
        t = gl.graphlet_last_timing()
        for k, v in t.items():
            if not isinstance(v, list):
                phase_sum[k] = phase_sum.get(k, 0) + v
        if counts is not None and c != counts:
            raise RuntimeError("counts changed between steps")
        counts = c
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms = dt / args.steps * 1e3
    timing = {k: v / args.steps for k, v in phase_sum.items()}
    log("[bench] phases: " + ", ".join(f"{k}={v:.3f}" for k, v in timing.items() if k.endswith("_ms")))
    name, roof = roofline_from_timing(timing, per_edge)
    roof["traffic"] = measured_traffic(roof["kernel"], args.workload)
    roof["l2_hit_rate"] = measured_traffic(roof["kernel"], args.workload, "l2_hit_rate")
    value = g.m / (ms / 1e3)
    res = {
        "metric": "edges/sec full k<=4 graphlet counts",
        "value": value,
        "unit": "edges/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int64/u128 (exact integer)",
        "data": "synthetic",
        "config": {"workload": args.workload, "n": g.n, "m": g.m, "csr_sha256": g.sha256(),
                   "params": params,
                   "output": "17 x u128 global counts" + (
                       " + 3 x int64[m] per-edge arrays" if per_edge else "")},
        "roofline": roof,
        "step_ms": {"min": min(step_ms), "median": sorted(step_ms)[len(step_ms) // 2],
                    "max": max(step_ms)},
        "h2d_ms": h2d_ms,
        "edges_per_s_incl_h2d": g.m / ((ms + h2d_ms) / 1e3),
        "phases_ms": {k: round(v, 3) for k, v in timing.items() if k.endswith("_ms")},
        "work": {k: timing[k] for k in ("clique_entries", "wedges_light", "wedges_heavy",
                                         "wedges_dense", "dense_hubs", "heavy_items")},
        "counts": [str(x) for x in counts],
    }
    st = stored_oracle({"rmat22": "rmat", "er": "er", "cl": "cl"}[args.workload])
    if st is not None and st.get("sha256") == g.sha256():
        res["matches_oracle"] = [int(x) for x in st["counts"]] == counts
        if not res["matches_oracle"]:
            raise SystemExit("counts differ from the stored oracle counts")
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (oracle, one core)...")
        res["cpu_baseline"] = cpu_baseline(g, {"rmat22": "rmat", "er": "er", "cl": "cl"}[
            args.workload], args.cpu_seconds)
    return res


def batch_alu_work(b, triangles):
    """Algorithmic work of the batched kernel over a batch, in 64-bit word
    operations (AND of two adjacency-row words and a popcount): per graph,
    W words per row times (edges [Step 1] + triangles [the 4-clique listing
    from each triangle's lowest edge, at most W words each] + vertex pairs
    of the 4-cycle pass [all pairs, or for a sparse graph the pairs two
    steps apart, plus the row unions that find them]), with the kernel's own
    dense / sparse choice (sum deg^2 + 2m < n^2 / 2 is sparse)."""
    import numpy as np
    import scipy.sparse as sp

    no, rp, col = b.node_off, b.row_ptr, b.col
    total = 0
    for gi in range(b.graphs):
        r0, r1 = int(no[gi]), int(no[gi + 1])
        n = r1 - r0
        e0, e1 = int(rp[r0]), int(rp[r1])
        nnz = e1 - e0
        w = (n + 63) // 64
        deg = np.diff(rp[r0:r1 + 1]).astype(np.int64)
        work = (nnz // 2 + int(triangles[gi])) * w
        if int((deg * deg).sum()) + nnz < n * n // 2:
            a = sp.csr_matrix((np.ones(nnz, np.int32), col[e0:e1], rp[r0:r1 + 1] - e0),
                              shape=(n, n))
            a2 = (a @ a).tocoo()
            work += int((a2.col > a2.row).sum()) * w
            work += int((deg * (w - ((np.arange(n) + 1) >> 6))).sum())
        else:
            work += n * (n - 1) // 2 * w
        total += work
    return total


def plan_device_ms(torch, plan, reps=5):
    """Device time of one replay, from events on the replay's stream."""
    st = torch.cuda.current_stream()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    best = float("inf")
    for _ in range(reps):
        a.record(st)
        plan.run(stream=st)
        b.record(st)
        b.synchronize()
        best = min(best, a.elapsed_time(b))
    return best


def run_batch(args, torch, gl):
    import graphgen.configs as C

    t0 = time.time()
    b = C.batch8192()
    log(f"[bench] generated batch: {b.graphs} graphs, {int(b.node_off[-1])} nodes, "
        f"{b.col.shape[0] // 2} edges in {time.time() - t0:.1f}s")
    dev = torch.device("cuda:0")
    no, rp, col = (torch.from_numpy(x).to(dev) for x in (b.node_off, b.row_ptr, b.col))
    out = torch.empty((b.graphs, 17), dtype=torch.int64, device=dev)
    # one-shot calls (plan, direct launches, no capture) for reference
    gl.graphlet_count_batched(no, rp, col, out=out)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(3):
        gl.graphlet_count_batched(no, rp, col, out=out)
    torch.cuda.synchronize()
    oneshot_ms = (time.perf_counter() - t0) / 3 * 1e3
    eager = out.clone()
    # the measured form: autotuned plan, persistent launch replayed as a HIP graph
    t0 = time.perf_counter()
    plan = gl.BatchPlan(no, rp, col, tune=True, out=out)
    tune_s = time.perf_counter() - t0
    info = plan.info()
    log(f"[bench] autotuned in {tune_s:.2f}s: {info}")
    for _ in range(args.warmup):
        plan.run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        plan.run()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / args.steps * 1e3
    if not torch.equal(out, eager):
        raise SystemExit("batched plan replay differs from the one-shot call")
    ms_dev = plan_device_ms(torch, plan)
    plan.close()
    # the kernel's roofline: 4 lane operations per word operation (two 32-bit
    # ANDs, two 32-bit popcounts), over the device time of one replay
    word_ops = batch_alu_work(b, out[:, 2].cpu().numpy())
    achieved = 4 * word_ops / (ms_dev / 1e3) / 1e12
    roof = {"bound": "alu", "achieved": round(achieved, 3), "peak": round(ALU_PEAK_TOPS, 2),
            "unit": "Tops/s (32-bit integer lane operations)",
            "frac": round(achieved / ALU_PEAK_TOPS, 4), "traffic": None, "kernel": "k_batched",
            "ops_per_launch": 4 * word_ops,
            "work_unit": "64-bit row-word AND + popcount = 4 lane operations; one replay "
                         "(every class launch) of the batch",
            "lds_bytes_per_word_op": 16}
    matches = None
    st = stored_oracle("batch8192")
    if st is not None and st.get("sha256") == b.sha256():
        import numpy as np

        with np.load(os.path.join(ROOT, "tests", "golden", st["counts_file"])) as z:
            matches = bool((out.cpu().numpy() == z["counts"]).all())
        if not matches:
            raise SystemExit("batched counts differ from the stored oracle counts")
    # baseline: one plain graphlet_count launch per graph, on a sample
    import numpy as np

    rng = np.random.default_rng(0)
    sample = rng.choice(b.graphs, size=min(args.per_graph_sample, b.graphs), replace=False)
    dev_graphs = []
    for i in sample:
        g = b.graph(int(i))
        dev_graphs.append((torch.from_numpy(g.row_ptr).to(dev), torch.from_numpy(g.col).to(dev), g.n))
    for rp1, col1, n1 in dev_graphs[:8]:
        gl.graphlet_count(rp1, col1, n1)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for rp1, col1, n1 in dev_graphs:
        gl.graphlet_count(rp1, col1, n1)
    torch.cuda.synchronize()
    per_graph_s = (time.perf_counter() - t1) / len(dev_graphs)
    log(f"[bench] batched {ms:.2f} ms for {b.graphs} graphs; per-graph launches "
        f"{per_graph_s * 1e3:.3f} ms/graph")
    cpu = None
    if not args.no_cpu_baseline:
        import oracle

        order = rng.permutation(b.graphs)
        done, t0 = 0, time.perf_counter()
        while time.perf_counter() - t0 < args.cpu_seconds / 2 and done < b.graphs:
            oracle.identity_route(b.graph(int(order[done])))
            done += 1
        dt = time.perf_counter() - t0
        cpu = {"value": done / dt, "unit": "graphs/s", "cores": 1, "kind": "oracle",
               "route": "oracle.identity_route per graph",
               "sample": f"{done} uniformly sampled graphs of the batch, {dt:.1f} s",
               "host": host_cpu()}
    return {
        "metric": "batched graphs/sec", "value": b.graphs / (ms / 1e3), "unit": "graphs/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "int64 (exact integer)", "data": "synthetic",
        "config": {"workload": "batch8192", "graphs": b.graphs, "csr_sha256": b.sha256(),
                   "params": C.BATCH},
        "plan": info, "tune_s": tune_s, "device_ms_per_step": ms_dev, "roofline": roof,
        "one_shot_graphs_per_s": b.graphs / (oneshot_ms / 1e3),
        "per_graph_launches": {"graphs_per_s": 1.0 / per_graph_s,
                               "sample": f"{len(dev_graphs)} graphs of the batch, one "
                                         "graphlet_count call each, CSR resident"},
        "speedup_vs_per_graph": (b.graphs / (ms / 1e3)) * per_graph_s,
        "matches_oracle": matches,
        "cpu_baseline": cpu,
    }


def serve_trace(gl, graphs, trace, slots, budget, want=None, batch_lane=True):
    """Replays (arrival_s, pool index) against a server; returns its stats.
    With `want` (the oracle's counts of each pool graph), every result is
    checked against it."""
    with gl.Server(budget_bytes=budget, slots=slots, batch_lane=batch_lane) as srv:
        t0 = time.perf_counter()
        ids = []
        for at, gi in trace:
            delay = at - (time.perf_counter() - t0)
            if delay > 0:
                time.sleep(delay)
            g = graphs[gi]
            ids.append(srv.submit(g.n, g.row_ptr, g.col))
        for i, (_, gi) in zip(ids, trace):
            counts, _ = srv.wait(i)
            if want is not None and counts != want[gi]:
                raise SystemExit(f"served counts of pool graph {gi} differ from the oracle's")
        st = srv.stats()
    return st


def run_serve(args, torch, gl):
    """Poisson arrivals at 200 req/s of graphs with m log-uniform in [1e3, 2e6]
    (half Chung-Lu exponent 2.3, half ER, mean degree 10).  A pool of
    distinct graphs drawn from the same trace distribution stands in for the
    request stream (each request is counted independently, so repeats of a
    pool graph cost the same as new graphs).  Served: 4 slots (streams) with
    admission by device-memory footprint, and the batch lane for graphs of at
    most 1024 vertices.  Baseline: the same trace through one slot and no
    batch lane, i.e. plain per-request launches in arrival order."""
    import graphgen.configs as C

    nreq = args.requests
    pool_n = min(args.pool, nreq)
    t0 = time.time()
    reqs, graphs = C.serve_pool(nreq, pool_n)
    log(f"[bench] serve pool: {pool_n} graphs, {sum(g.m for g in graphs)} edges "
        f"in {time.time() - t0:.1f}s; {nreq} requests")
    trace = [(reqs[i][0], i % pool_n) for i in range(nreq)]
    budget = 64 << 30
    want = None
    st = stored_oracle("serve_pool")
    if st is not None and len(st["graphs"]) == pool_n and all(
            g.sha256() == s["sha256"] for g, s in zip(graphs, st["graphs"])):
        want = [[int(x) for x in s["counts"]] for s in st["graphs"]]
    # warm up the library and the stream-ordered allocator
    serve_trace(gl, graphs, [(0.0, i) for i in range(min(8, pool_n))], 4, budget)
    served = serve_trace(gl, graphs, trace, 4, budget, want)
    log(f"[bench] served: {served['graphs_per_s']:.1f} graphs/s p50 {served['p50_ms']:.2f} ms "
        f"p99 {served['p99_ms']:.2f} ms")
    plain = serve_trace(gl, graphs, trace, 1, budget, want, batch_lane=False)
    log(f"[bench] per-request plain: {plain['graphs_per_s']:.1f} graphs/s "
        f"p50 {plain['p50_ms']:.2f} ms p99 {plain['p99_ms']:.2f} ms")
    # saturated: every request at time 0
    sat = serve_trace(gl, graphs, [(0.0, i % pool_n) for i in range(nreq)], 4, budget)
    sat1 = serve_trace(gl, graphs, [(0.0, i % pool_n) for i in range(nreq)], 1, budget,
                       batch_lane=False)
    log(f"[bench] saturated: served {sat['graphs_per_s']:.1f} graphs/s, plain "
        f"{sat1['graphs_per_s']:.1f} graphs/s")
    keep = ("completed", "failed", "p50_ms", "p99_ms", "mean_ms", "graphs_per_s", "edges_per_s",
            "bytes_peak", "elapsed_s", "batches", "batched")
    return {
        "metric": "served graphs/sec (Poisson 200 req/s) with p50/p99 latency",
        "value": served["graphs_per_s"], "unit": "graphs/s", "n_gpus": 1,
        "steps": nreq, "warmup": 8, "ms_per_step": served["mean_ms"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u128 (exact integer)", "data": "synthetic",
        "config": {"workload": "serve", "requests": nreq, "pool_graphs": pool_n,
                   "params": C.SERVE, "slots": 4, "budget_bytes": budget},
        "p50_ms": served["p50_ms"], "p99_ms": served["p99_ms"],
        "served": {k: served[k] for k in keep},
        "per_request_plain": {k: plain[k] for k in keep},
        "saturated_served": {k: sat[k] for k in keep},
        "saturated_plain": {k: sat1[k] for k in keep},
        "matches_oracle": want is not None,
    }


def run_update(args, torch, gl):
    """Localized edge updates on R-MAT scale 22: each of `--requests` random
    edges (half of them at the 64 highest-degree vertices) is deleted and
    inserted again with graphlet_update_edge; the counts must come back to
    the full count's.  Latency per update against one full recount."""
    import numpy as np

    import graphgen.configs as C

    g = C.rmat22()
    dev = torch.device("cuda:0")
    rp = torch.from_numpy(g.row_ptr).to(dev)
    col = torch.from_numpy(g.col).to(dev)
    t0 = time.perf_counter()
    base = gl.graphlet_count(rp, col, g.n)
    torch.cuda.synchronize()
    full_ms = (time.perf_counter() - t0) * 1e3
    rng = np.random.default_rng(7)
    deg = np.diff(g.row_ptr)
    hubs = np.argsort(-deg)[:64]
    k = max(2, args.requests // 10)
    lat = []
    pairs_done = []
    for i in range(k):
        u = int(hubs[i % 64]) if i % 2 else int(rng.choice(np.nonzero(deg)[0]))
        v = int(g.col[g.row_ptr[u] + rng.integers(deg[u])])
        # the graph without (u, v), as a CSR on the device
        keep = np.ones(g.col.shape[0], bool)
        a, b = g.row_ptr[u], g.row_ptr[v]
        keep[a + np.searchsorted(g.col[a:g.row_ptr[u + 1]], v)] = False
        keep[b + np.searchsorted(g.col[b:g.row_ptr[v + 1]], u)] = False
        rp2 = g.row_ptr.copy()
        rp2[u + 1:] -= 1
        rp2[v + 1:] -= 1
        rp_d, col_d = torch.from_numpy(rp2).to(dev), torch.from_numpy(g.col[keep]).to(dev)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        less = gl.graphlet_update_edge(rp, col, g.n, u, v, False, base)
        t2 = time.perf_counter()
        back = gl.graphlet_update_edge(rp_d, col_d, g.n, u, v, True, less)
        t3 = time.perf_counter()
        if back != base:
            raise SystemExit("edge update round trip differs from the full count")
        lat += [(t2 - t1) * 1e3, (t3 - t2) * 1e3]
        pairs_done.append((u, v))
    lat = np.array(lat)
    log(f"[bench] {len(lat)} updates: p50 {np.percentile(lat, 50):.3f} ms, "
        f"p99 {np.percentile(lat, 99):.3f} ms; full recount {full_ms:.1f} ms")
    # the same deletions and re-insertions served against the graph kept
    # resident in the server (counts by the localized update, then the CSR
    # rewritten into its spare buffer); latency = completion - submission
    pairs = pairs_done
    with gl.Server(budget_bytes=64 << 30, slots=2) as srv:
        gid = srv.register(g.n, g.row_ptr, g.col)
        if srv.wait(gid)[0] != base:
            raise SystemExit("resident registration differs from the full count")
        slat = []
        for u, v in pairs:
            less, l1 = srv.wait(srv.update(gid, u, v, False))
            back, l2 = srv.wait(srv.update(gid, u, v, True))
            if back != base:
                raise SystemExit("served update round trip differs from the full count")
            slat += [l1, l2]
        srv.unregister(gid)
    slat = np.array(slat)
    log(f"[bench] {len(slat)} served updates: p50 {np.percentile(slat, 50):.3f} ms, "
        f"p99 {np.percentile(slat, 99):.3f} ms")
    return {
        "metric": "edge updates/sec (R-MAT s22, localized recount)",
        "value": 1e3 / float(lat.mean()), "unit": "updates/s", "n_gpus": 1,
        "steps": int(len(lat)), "warmup": 0, "ms_per_step": float(lat.mean()),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u128 (exact integer)", "data": "synthetic",
        "config": {"workload": "update", "graph": "rmat22", "n": g.n, "m": g.m,
                   "edges": "half uniform, half at the 64 highest-degree vertices"},
        "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
        "full_recount_ms": full_ms,
        "served_resident": {"updates": int(len(slat)), "p50_ms": float(np.percentile(slat, 50)),
                            "p99_ms": float(np.percentile(slat, 99)),
                            "includes": "queueing, localized count update and CSR rewrite"},
    }


def vertex_roofline(g, ms):
    """k_vertex_counts: one wave per vertex reads its list (col2 4 B, the
    twin position 4 B for the lower half), the edge's five per-edge words
    (|Tri| 4 B, K4 / C4 / D / B 8 B each) and the neighbour's degree, triangle
    and degree-sum words (4 + 8 + 8 B); per vertex its row bounds, lower
    count, order, own sums and the 17 x 8 B output."""
    nnz = 2 * g.m
    nbytes = nnz * (4 + 4 + 32 + 20) + (nnz // 2) * 4 + g.n * (8 + 4 + 4 + 20 + 136)
    achieved = nbytes / (ms / 1e3) / 1e9 if ms > 0 else 0.0
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
            "kernel": "k_vertex_counts", "phase_ms": round(ms, 3), "bytes_per_launch": nbytes,
            "work_unit": "per adjacency entry 60 B + 4 B per lower entry, per vertex 172 B"}


def run_vertex(args, torch, gl):
    """Per-vertex counts (17 per vertex, graphlet_count_vertex) of R-MAT
    scale 22; vertices/s of the whole call, the per-vertex kernel's own
    device time, and the sum rule (each k-node class seen k times) checked
    on the device against the global counts."""
    import graphgen.configs as C

    g = C.rmat22()
    dev = torch.device("cuda:0")
    rp = torch.from_numpy(g.row_ptr).to(dev)
    col = torch.from_numpy(g.col).to(dev)
    ws_bytes = gl.graphlet_workspace_size(rp, col, g.n, per_edge=2)
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device=dev)
    out = torch.empty((17, g.n), dtype=torch.uint64, device=dev)
    log(f"[bench] vertex: workspace {ws_bytes / 2**30:.2f} GiB")
    gl.graphlet_timing_enable(True)
    counts = None
    for i in range(args.warmup):
        counts, V = gl.graphlet_count_vertex(rp, col, g.n, workspace=ws, out=out)
        log(f"[bench] warmup {i} done")
    torch.cuda.synchronize()
    phase_sum = {}
    t0 = time.perf_counter()
    for _ in range(args.steps):
        c, V = gl.graphlet_count_vertex(rp, col, g.n, workspace=ws, out=out)
        for k, v in gl.graphlet_last_timing().items():
            if not isinstance(v, list):
                phase_sum[k] = phase_sum.get(k, 0) + v
        if counts is not None and c != counts:
            raise RuntimeError("counts changed between steps")
        counts = c
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / args.steps * 1e3
    timing = {k: v / args.steps for k, v in phase_sum.items()}
    k_of = [2, 2, 3, 3, 3, 3] + [4] * 11
    Vi = V.view(torch.int64)
    lo = (Vi & 0xFFFFFFFF).sum(dim=1).tolist()
    hi = ((Vi >> 32) & 0xFFFFFFFF).sum(dim=1).tolist()
    for cl in range(17):
        if lo[cl] + (hi[cl] << 32) != k_of[cl] * counts[cl]:
            raise SystemExit(f"per-vertex sum rule fails for class {cl}")
    log(f"[bench] vertex: {ms:.1f} ms per call, kernel {timing['vertex_ms']:.3f} ms")
    return {
        "metric": "vertices/sec per-vertex k<=4 graphlet counts (R-MAT s22)",
        "value": g.n / (ms / 1e3), "unit": "vertices/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u64 per vertex, u128 global (exact integer)",
        "data": "synthetic",
        "config": {"workload": "vertex", "graph": "rmat22", "n": g.n, "m": g.m,
                   "csr_sha256": g.sha256(), "output": "17 x u64 per vertex + 17 x u128"},
        "edges_per_s": g.m / (ms / 1e3),
        "roofline": vertex_roofline(g, timing["vertex_ms"]),
        "phases_ms": {k: round(v, 3) for k, v in timing.items() if k.endswith("_ms")},
    }


def run_batch_vertex(args, torch, gl):
    """Per-vertex counts of every vertex of the 8192-graph batch
    (graphlet_batch_vertex, one call per step); graphs/s and vertices/s, the
    sum rule (per graph, each k-node class seen k times over its vertices)
    checked against the batched global counts, and per-graph
    graphlet_count_vertex calls on a sample as the unbatched alternative."""
    import graphgen.configs as C
    import numpy as np

    b = C.batch8192()
    dev = torch.device("cuda:0")
    no, rp, col = (torch.from_numpy(x).to(dev) for x in (b.node_off, b.row_ptr, b.col))
    nv = int(b.node_off[-1])
    out = torch.empty((nv, 17), dtype=torch.uint64, device=dev)
    for _ in range(args.warmup):
        gl.graphlet_batch_vertex(no, rp, col, out=out)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        gl.graphlet_batch_vertex(no, rp, col, out=out)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / args.steps * 1e3
    counts = gl.graphlet_count_batched(no, rp, col).cpu().numpy()
    V = out.cpu().numpy().astype(np.int64)
    gid = np.repeat(np.arange(b.graphs), np.diff(b.node_off))
    per_graph = np.zeros((b.graphs, 17), np.int64)
    np.add.at(per_graph, gid, V)
    k_of = np.array([2, 2, 3, 3, 3, 3] + [4] * 11)
    if not (per_graph == counts * k_of).all():
        raise SystemExit("batched per-vertex sum rule fails")
    rng = np.random.default_rng(0)
    sample = rng.choice(b.graphs, size=min(args.per_graph_sample, b.graphs), replace=False)
    dev_graphs = []
    for i in sample:
        g = b.graph(int(i))
        dev_graphs.append((torch.from_numpy(g.row_ptr).to(dev), torch.from_numpy(g.col).to(dev), g.n))
    for rp1, col1, n1 in dev_graphs[:8]:
        gl.graphlet_count_vertex(rp1, col1, n1)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for rp1, col1, n1 in dev_graphs:
        gl.graphlet_count_vertex(rp1, col1, n1)
    torch.cuda.synchronize()
    per_graph_s = (time.perf_counter() - t1) / len(dev_graphs)
    log(f"[bench] batched per-vertex {ms:.2f} ms for {b.graphs} graphs ({nv} vertices); "
        f"per-graph calls {per_graph_s * 1e3:.3f} ms/graph")
    return {
        "metric": "batched graphs/sec, per-vertex counts", "value": b.graphs / (ms / 1e3),
        "unit": "graphs/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u64 (exact integer)", "data": "synthetic",
        "config": {"workload": "batch8192_vertex", "graphs": b.graphs, "vertices": nv,
                   "csr_sha256": b.sha256(), "params": C.BATCH},
        "vertices_per_s": nv / (ms / 1e3),
        "per_graph_calls": {"graphs_per_s": 1.0 / per_graph_s,
                            "sample": f"{len(dev_graphs)} graphs of the batch, one "
                                      "graphlet_count_vertex call each, CSR resident"},
        "speedup_vs_per_graph": (b.graphs / (ms / 1e3)) * per_graph_s,
    }


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="rmat22",
                    choices=["rmat22", "er", "cl", "batch", "batch_vertex", "serve", "update",
                             "vertex"])
    ap.add_argument("--requests", type=int, default=1000, help="serve: trace length")
    ap.add_argument("--pool", type=int, default=96, help="serve: distinct graphs")
    ap.add_argument("--per-graph-sample", type=int, default=256,
                    help="batch: graphs timed with one plain launch each")
    ap.add_argument("--cpu-seconds", type=float, default=6.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="rmat22: skip the batched and serving parts of the metric")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only copy a 1 GiB device buffer 3 times (known bytes per dispatch, "
                         "to scale hardware byte counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path",
              file=sys.stderr)
        sys.exit(2)
    import torch

    import paper_1506_04322_amd as gl

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(3)
    gl.load()
    if args.copy_calibration:
        src = torch.ones(1 << 28, dtype=torch.int32, device="cuda:0")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / 3
        print(json.dumps({"copy_bytes_read": 1 << 30, "copy_bytes_written": 1 << 30,
                          "copy_GBps": 2 * (1 << 30) / dt / 1e9}), flush=True)
        return
    if args.workload == "batch":
        res = run_batch(args, torch, gl)
    elif args.workload == "serve":
        res = run_serve(args, torch, gl)
    elif args.workload == "update":
        res = run_update(args, torch, gl)
    elif args.workload == "vertex":
        res = run_vertex(args, torch, gl)
    elif args.workload == "batch_vertex":
        res = run_batch_vertex(args, torch, gl)
    else:
        res = run_single(args, torch, gl)
        if args.workload == "rmat22" and not args.no_extras:
            # the other two parts of the metric, compact: batched graphs/s
            # against per-graph launches, served graphs/s and p50 / p99
            # against per-request plain launches
            b = run_batch(args, torch, gl)
            res["batched"] = {k: b[k] for k in (
                "metric", "value", "unit", "ms_per_step", "device_ms_per_step",
                "one_shot_graphs_per_s", "per_graph_launches", "speedup_vs_per_graph",
                "matches_oracle", "plan", "cpu_baseline", "roofline")}
            res["batched"]["config"] = b["config"]
            sv = run_serve(args, torch, gl)
            res["serve"] = {k: sv[k] for k in (
                "metric", "value", "unit", "p50_ms", "p99_ms", "served", "per_request_plain",
                "saturated_served", "saturated_plain", "matches_oracle", "config")}
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
