"""Writes tests/golden/configs.json: oracle counts of the seeded workloads.

Calls only the CPU oracle (the identity route, exact at any size) on the
graphs of graphgen.configs, and stores each 17-vector with the SHA-256 of the
CSR it was computed on, so a test can tell a changed input from a wrong
count.  Slow by design (single-threaded plain C): minutes for the power-law
graph, tens of minutes for R-MAT scale 22.

usage: python tests/golden/make_golden.py [er] [cl] [rmat]
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import graphgen.configs as C  # noqa: E402
import oracle  # noqa: E402

OUT = os.path.join(HERE, "configs.json")


def main(which):
    data = {}
    if os.path.exists(OUT):
        with open(OUT) as f:
            data = json.load(f)
    builders = {"er": C.er, "cl": C.cl, "rmat": C.rmat22}
    for name in which:
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
        }
        print(name, g.n, g.m, dt, counts, flush=True)
        with open(OUT, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)


if __name__ == "__main__":
    main(sys.argv[1:] or ["er", "cl", "rmat"])
