"""The five synthetic workloads, with fixed seeds.

The paper measures real networks (Section 5, Table 2), which are not
available here; these seeded stand-ins have the shapes the benchmark calls
for.  Each builder returns the same graph on every host.
"""
from __future__ import annotations

import math

import numpy as np

from . import batch, chung_lu, er_gnm, rmat

# 1: Erdos-Renyi G(n = 2000, m = 20000)
ER = dict(n=2000, m=20000, seed=1)
# 2: Chung-Lu power law, 1M nodes, expected-degree exponent 2.1; ball dropping
#    with weights (i + 13)^(-1/1.1) and 10.9M balls gives m ~ 1.0e7, max deg ~ 5e4
CL = dict(n=1_000_000, beta=2.1, i0=13.0, balls=10_900_000, seed=2)
# 3: R-MAT scale 22, edge factor 16, (a, b, c, d) = (0.57, 0.19, 0.19, 0.05)
RMAT = dict(scale=22, edge_factor=16, a=0.57, b=0.19, c=0.19, seed=3)
# 4: 8192 small graphs, n uniform in [20, 600]; 80% ER with density in
#    [0.02, 0.3], 20% torus random geometric graphs of mean degree 8
BATCH = dict(G=8192, nmin=20, nmax=600, rho_min=0.02, rho_max=0.3, rgg_frac=0.2, rgg_deg=8.0,
             seed=4)
# 5: serving: Poisson arrivals at 200 req/s, m log-uniform in [1e3, 2e6],
#    half Chung-Lu (exponent 2.3), half ER, mean degree 10 (n = m / 5)
SERVE = dict(rate=200.0, m_min=1_000, m_max=2_000_000, beta=2.3, mean_degree=10.0, seed=5)


def er():
    return er_gnm(ER["n"], ER["m"], ER["seed"])


def cl():
    return chung_lu(CL["n"], CL["beta"], CL["i0"], CL["balls"], CL["seed"])


def rmat22():
    return rmat(RMAT["scale"], RMAT["edge_factor"], RMAT["a"], RMAT["b"], RMAT["c"], RMAT["seed"])


def batch8192(G: int | None = None):
    p = BATCH
    return batch(G if G is not None else p["G"], p["nmin"], p["nmax"], p["rho_min"], p["rho_max"],
                 p["rgg_frac"], p["rgg_deg"], p["seed"])


def serve_requests(count: int, seed: int | None = None):
    """Request trace: (arrival_time_s, kind, n, m, graph_seed) for `count` requests."""
    p = SERVE
    rng = np.random.default_rng(p["seed"] if seed is None else seed)
    gaps = rng.exponential(1.0 / p["rate"], size=count)
    t = np.cumsum(gaps) - gaps[0]
    lm = rng.uniform(math.log(p["m_min"]), math.log(p["m_max"]), size=count)
    ms = np.exp(lm).astype(np.int64)
    kinds = rng.integers(0, 2, size=count)  # 0 ER, 1 Chung-Lu
    seeds = rng.integers(1, 2**62, size=count)
    out = []
    for i in range(count):
        m = int(ms[i])
        n = max(16, int(round(2 * m / p["mean_degree"])))
        out.append((float(t[i]), "cl" if kinds[i] else "er", n, m, int(seeds[i])))
    return out


def serve_graph(kind: str, n: int, m: int, seed: int):
    """One request's graph.  Chung-Lu drops repeats, so it draws ~10% extra balls."""
    if kind == "er":
        return er_gnm(n, m, seed)
    return chung_lu(n, SERVE["beta"], 1.0, int(m * 1.1), seed)


# The serving benchmark replays a trace of SERVE_REQUESTS requests over a
# pool of the graphs of its first SERVE_POOL requests.
SERVE_REQUESTS = 1000
SERVE_POOL = 96


def serve_pool(requests: int = SERVE_REQUESTS, pool: int = SERVE_POOL):
    """(trace, graphs): the request trace and the distinct graphs of its
    first `pool` requests, the pool the serving benchmark replays."""
    reqs = serve_requests(requests)
    graphs = [serve_graph(k, n, m, sd) for (_, k, n, m, sd) in reqs[:min(pool, requests)]]
    return reqs, graphs
