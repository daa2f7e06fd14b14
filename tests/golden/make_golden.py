"""Writes the stored oracle counts of the seeded workloads.

Calls only the CPU oracle (the identity route, exact at any size) on the
graphs of graphgen.configs, and stores each result with the SHA-256 of the
CSR it was computed on, so a test can tell a changed input from a wrong
count.  Slow by design (single-threaded plain C): minutes for the power-law
graph, tens of minutes for R-MAT scale 22, about a minute and a half for the
8192 small graphs.

  configs.json          er, cl, rmat: 17-vector per graph; batch8192: the
                        batch CSR hash and the hash of the count matrix;
                        serve_pool: the 96 distinct graphs of the serving
                        trace, each with its parameters, hash and 17-vector
  batch8192_counts.npz  int64 [8192, 17], row i the counts of graph i

usage: python tests/golden/make_golden.py [er] [cl] [rmat] [batch] [serve]
"""
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import graphgen.configs as C  # noqa: E402
import oracle  # noqa: E402

OUT = os.path.join(HERE, "configs.json")
BATCH_NPZ = os.path.join(HERE, "batch8192_counts.npz")


def host_cpu() -> dict:
    """The CPU the oracle ran on (its times are single-threaded)."""
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"cpu_model": model, "nproc": os.cpu_count(), "threads_used": 1}


def matrix_sha256(a: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(a, dtype="<i8").tobytes()).hexdigest()


def single(name, data):
    builders = {"er": C.er, "cl": C.cl, "rmat": C.rmat22}
    g = builders[name]()
    t0 = time.time()
    counts = oracle.identity_route(g)
    dt = time.time() - t0
    data[name] = {
        "n": g.n,
        "m": g.m,
        "sha256": g.sha256(),
        "counts": [str(c) for c in counts],
        "oracle_seconds": round(dt, 1),
        "route": "oracle.identity_route",
        "host": host_cpu(),
    }
    print(name, g.n, g.m, dt, counts, flush=True)


def batch(data):
    b = C.batch8192()
    t0 = time.time()
    out = np.zeros((b.graphs, 17), np.int64)
    for i in range(b.graphs):
        c = oracle.identity_route(b.graph(i))
        assert all(0 <= x < 2**63 for x in c)
        out[i] = c
    dt = time.time() - t0
    np.savez_compressed(BATCH_NPZ, counts=out)
    data["batch8192"] = {
        "graphs": b.graphs,
        "sha256": b.sha256(),
        "counts_file": os.path.basename(BATCH_NPZ),
        "counts_sha256": matrix_sha256(out),
        "oracle_seconds": round(dt, 1),
        "route": "oracle.identity_route per graph",
        "host": host_cpu(),
    }
    print("batch8192", b.graphs, dt, flush=True)


def serve_pool(data):
    reqs, graphs = C.serve_pool()
    pool = []
    t0 = time.time()
    for (_, kind, n, m, seed), g in zip(reqs, graphs):
        counts = oracle.identity_route(g)
        pool.append({"kind": kind, "n": n, "m_target": m, "seed": seed, "m": g.m,
                     "sha256": g.sha256(), "counts": [str(c) for c in counts]})
    dt = time.time() - t0
    data["serve_pool"] = {"graphs": pool, "oracle_seconds": round(dt, 1),
                          "route": "oracle.identity_route per graph", "host": host_cpu(),
                          "trace": "graphgen.configs.serve_pool(): the first %d of %d requests" %
                                   (C.SERVE_POOL, C.SERVE_REQUESTS)}
    print("serve_pool", len(pool), sum(p["m"] for p in pool), dt, flush=True)


def main(which):
    data = {}
    if os.path.exists(OUT):
        with open(OUT) as f:
            data = json.load(f)
    for name in which:
        if name == "batch":
            batch(data)
        elif name == "serve":
            serve_pool(data)
        else:
            single(name, data)
        with open(OUT, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)


if __name__ == "__main__":
    main(sys.argv[1:] or ["er", "cl", "rmat", "batch", "serve"])
