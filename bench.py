#!/usr/bin/env python3
"""Benchmark: exact k <= 4 graphlet counts on one MI355X.

Default workload: R-MAT scale 22 (edge factor 16, a,b,c,d = .57,.19,.19,.05,
64.2M undirected edges after symmetrising and deduplicating), full 17-class
counts, CSR resident in HBM before the timed region.  One step = one
graphlet_count call (prepass, Steps 1-4, result on the host).

Prints one JSON line (the last line of stdout).  Other workloads:
  --workload er | cl | batch
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, GB/s


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_baseline(g, seconds: float, seed: int = 0):
    """The oracle's per-edge route (|Tri_e|, 4-cliques, induced 4-cycles per
    edge, literally) on a random sample of the same graph's edges, run for
    about `seconds` on one host core; edges/s."""
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
    return {"value": done / dt, "unit": "edges/s", "cores": 1, "kind": "oracle",
            "sample": f"{done} uniformly sampled edges of the same graph, per-edge oracle "
                      f"(|Tri_e|, 4-cliques and induced 4-cycles by definition), {dt:.1f} s"}


def roofline_from_timing(t: dict):
    """Dominant counting phase, its algorithmic bytes (4 B per adjacency entry
    the phase must read) over its measured device time."""
    phases = {
        "cyc_heavy": (t["cyc_heavy_ms"], 4 * t["wedges_heavy"],
                      "k_c4_heavy", "wedges of heavy vertices x 4 B"),
        "cyc_light": (t["cyc_light_ms"], 4 * t["wedges_light"],
                      "k_c4_light", "wedges of light vertices x 4 B"),
        "cliques": (t["cliques_ms"], 4 * t["clique_entries"],
                    "k_tk_lds/k_tk_global", "upper-list entries scanned x 4 B"),
    }
    name = max(phases, key=lambda k: phases[k][0])
    ms, nbytes, kern, unit = phases[name]
    achieved = nbytes / (ms / 1e3) / 1e9 if ms > 0 else 0.0
    return name, {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                  "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                  "kernel": kern, "phase_ms": round(ms, 3), "bytes_per_launch": nbytes,
                  "work_unit": unit}


def run_single(args, torch, gl):
    import graphgen.configs as C

    builders = {"rmat22": (C.rmat22, C.RMAT), "er": (C.er, C.ER), "cl": (C.cl, C.CL)}
    build, params = builders[args.workload]
    t0 = time.time()
    g = build()
    log(f"[bench] generated {args.workload}: n={g.n} m={g.m} in {time.time() - t0:.1f}s")
    dev = torch.device("cuda:0")
    rp = torch.from_numpy(g.row_ptr).to(dev)
    col = torch.from_numpy(g.col).to(dev)
    ws_bytes = gl.graphlet_workspace_size(rp, col, g.n)
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device=dev)
    log(f"[bench] workspace {ws_bytes / 2**30:.2f} GiB")
    gl.graphlet_timing_enable(True)
    counts = None
    for i in range(args.warmup):
        counts = gl.graphlet_count(rp, col, g.n, workspace=ws)
        log(f"[bench] warmup {i} done")
    torch.cuda.synchronize()
    phase_sum = {}
    t0 = time.perf_counter()
    for i in range(args.steps):
        c = gl.graphlet_count(rp, col, g.n, workspace=ws)
        t = gl.graphlet_last_timing()
        for k, v in t.items():
            phase_sum[k] = phase_sum.get(k, 0) + v
        if counts is not None and c != counts:
            raise RuntimeError("counts changed between steps")
        counts = c
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms = dt / args.steps * 1e3
    timing = {k: v / args.steps for k, v in phase_sum.items()}
    log("[bench] phases: " + ", ".join(f"{k}={v:.3f}" for k, v in timing.items() if k.endswith("_ms")))
    name, roof = roofline_from_timing(timing)
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
                   "params": params, "output": "17 x u128 global counts"},
        "roofline": roof,
        "phases_ms": {k: round(v, 3) for k, v in timing.items() if k.endswith("_ms")},
        "work": {k: timing[k] for k in ("clique_entries", "wedges_light", "wedges_heavy")},
        "counts": [str(x) for x in counts],
    }
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (oracle, one core)...")
        res["cpu_baseline"] = cpu_baseline(g, args.cpu_seconds)
    return res


def run_batch(args, torch, gl):
    import graphgen.configs as C

    t0 = time.time()
    b = C.batch8192()
    log(f"[bench] generated batch: {b.graphs} graphs, {int(b.node_off[-1])} nodes, "
        f"{b.col.shape[0] // 2} edges in {time.time() - t0:.1f}s")
    dev = torch.device("cuda:0")
    no, rp, col = (torch.from_numpy(x).to(dev) for x in (b.node_off, b.row_ptr, b.col))
    out = torch.empty((b.graphs, 17), dtype=torch.int64, device=dev)
    for _ in range(args.warmup):
        gl.graphlet_count_batched(no, rp, col, out=out)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        gl.graphlet_count_batched(no, rp, col, out=out)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / args.steps * 1e3
    return {
        "metric": "batched graphs/sec", "value": b.graphs / (ms / 1e3), "unit": "graphs/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "int64 (exact integer)", "data": "synthetic",
        "config": {"workload": "batch8192", "graphs": b.graphs, "csr_sha256": b.sha256(),
                   "params": C.BATCH},
    }


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="rmat22", choices=["rmat22", "er", "cl", "batch"])
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(the design for sharding is described in DESIGN.md)", file=sys.stderr)
        sys.exit(2)
    import torch

    import paper_1506_04322_amd as gl

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(3)
    gl.load()
    if args.workload == "batch":
        res = run_batch(args, torch, gl)
    else:
        res = run_single(args, torch, gl)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
