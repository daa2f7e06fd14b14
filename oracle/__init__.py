"""CPU oracle for graphlet counts (test infrastructure only).

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The GPU library never does, and the
two share no code: the C source here is compiled on its own with gcc.

Routes (see oracle.c for the definitions each one writes out):
  bruteforce(g)        every 2/3/4-subset classified by Table 1 (n <= ~300)
  identity_route(g)    non-induced counts inverted, exact at any size
  per_edge(g, edges)   |Tri_e|, 4-cliques and induced 4-cycles through e,
                       literally, one edge at a time
  bruteforce_edge4     4-cliques / 4-cycles through e by subset enumeration
  vertex_bruteforce    per-vertex counts: every subset credited to its members
  vertex_by_deletion   per-vertex counts as g(G) - g(G - v) via identity_route
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

NAMES = ["g2_1", "g2_2", "g3_1", "g3_2", "g3_3", "g3_4"] + [f"g4_{i}" for i in range(1, 12)]


class _U128(ctypes.Structure):
    _fields_ = [("lo", ctypes.c_uint64), ("hi", ctypes.c_uint64)]


def build() -> str:
    """Compile the oracle with gcc (plain C, -O2)."""
    cmd = ["gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", "-o", _LIB + ".tmp", _SRC]
    subprocess.run(cmd, check=True)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        I64 = ctypes.c_int64
        lib.oracle_check_csr.argtypes = [I64, P, P]
        lib.oracle_check_csr.restype = ctypes.c_int
        for f in (lib.oracle_bruteforce, lib.oracle_identity_route):
            f.argtypes = [I64, P, P, ctypes.POINTER(_U128)]
            f.restype = ctypes.c_int
        lib.oracle_per_edge.argtypes = [I64, P, P, I64, P, P, P, P, P]
        lib.oracle_per_edge.restype = ctypes.c_int
        lib.oracle_bruteforce_edge4.argtypes = [I64, P, P, I64, P, P, P, P]
        lib.oracle_bruteforce_edge4.restype = ctypes.c_int
        lib.oracle_vertex_bruteforce.argtypes = [I64, P, P, P]
        lib.oracle_vertex_bruteforce.restype = ctypes.c_int
        lib.oracle_edge_local.argtypes = [I64, P, P, I64, P, P, P]
        lib.oracle_edge_local.restype = ctypes.c_int
        lib.oracle_edge_local_brute.argtypes = [I64, P, P, I64, P, P, P]
        lib.oracle_edge_local_brute.restype = ctypes.c_int
        lib.oracle_edges.argtypes = [I64, P, P, P, P]
        lib.oracle_edges.restype = I64
        lib.oracle_classify4.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int]
        lib.oracle_classify4.restype = ctypes.c_int
        _lib = lib
    return _lib


def _csr(g):
    rp = np.ascontiguousarray(g.row_ptr, dtype=np.int32)
    col = np.ascontiguousarray(g.col, dtype=np.int32)
    if col.size == 0:
        col = np.zeros(1, dtype=np.int32)
    return int(g.n), rp, col


def _counts(fn, g) -> list[int]:
    n, rp, col = _csr(g)
    out = (_U128 * 17)()
    rc = fn(n, rp.ctypes.data, col.ctypes.data, out)
    if rc != 0:
        raise ValueError(f"oracle rejected the graph (code {rc})")
    return [int(o.lo) | (int(o.hi) << 64) for o in out]


def check_csr(g) -> int:
    n, rp, col = _csr(g)
    return int(_load().oracle_check_csr(n, rp.ctypes.data, col.ctypes.data))


def bruteforce(g) -> list[int]:
    """17 induced-graphlet counts by enumerating every subset (definition)."""
    return _counts(_load().oracle_bruteforce, g)


def identity_route(g) -> list[int]:
    """17 induced-graphlet counts from non-induced counts (exact, any size)."""
    return _counts(_load().oracle_identity_route, g)


def classify4(edges: int, maxdeg: int, comps: int) -> int:
    """Table 1 row (0..10 for g4_1..g4_11) from (edges, Delta, |C|); -1 if none."""
    return int(_load().oracle_classify4(edges, maxdeg, comps))


def edges(g) -> tuple[np.ndarray, np.ndarray]:
    """Undirected edges (u < v) in canonical order: u ascending, then v."""
    n, rp, col = _csr(g)
    lib = _load()
    m = lib.oracle_edges(n, rp.ctypes.data, col.ctypes.data, None, None)
    eu = np.empty(max(m, 1), dtype=np.int32)
    ev = np.empty(max(m, 1), dtype=np.int32)
    lib.oracle_edges(n, rp.ctypes.data, col.ctypes.data, eu.ctypes.data, ev.ctypes.data)
    return eu[:m], ev[:m]


# number of vertices of each of the 17 classes (the order of NAMES)
CLASS_K = [2, 2, 3, 3, 3, 3] + [4] * 11


def vertex_bruteforce(g) -> np.ndarray:
    """[n, 17] int64: k-subsets containing each vertex, by induced class (definition)."""
    n, rp, col = _csr(g)
    out = np.zeros((max(n, 1), 17), dtype=np.int64)
    rc = _load().oracle_vertex_bruteforce(n, rp.ctypes.data, col.ctypes.data, out.ctypes.data)
    if rc != 0:
        raise ValueError(f"per-vertex brute force rejected the graph (code {rc})")
    return out[:n]


def delete_vertex(g, v: int):
    """G - v: the induced subgraph on V minus {v}, ids above v shifted down by one."""
    rp = np.asarray(g.row_ptr, dtype=np.int64)
    col = np.asarray(g.col, dtype=np.int64)
    n = int(g.n)
    deg = np.diff(rp)
    src = np.repeat(np.arange(n, dtype=np.int64), deg)
    keep = (src != v) & (col != v)
    src, dst = src[keep], col[keep]
    src = src - (src > v)
    dst = dst - (dst > v)
    cnt = np.bincount(src, minlength=n - 1) if n > 1 else np.zeros(0, dtype=np.int64)
    rp2 = np.zeros(n, dtype=np.int32)
    if n > 1:
        rp2[1:] = np.cumsum(cnt)
    # rows stay sorted: the shift keeps the order of the remaining ids
    return _Graph(n - 1, rp2, dst.astype(np.int32))


class _Graph:
    def __init__(self, n, row_ptr, col):
        self.n, self.row_ptr, self.col = n, row_ptr, col


def vertex_by_deletion(g, vertices=None) -> np.ndarray:
    """[len(vertices), 17] uint64 per-vertex counts as g_c(G) - g_c(G - v).

    A k-subset of class c either contains v or survives in G - v unchanged, so
    the difference of the two global count vectors (both from
    identity_route, which knows nothing of vertices) is the per-vertex
    count.  Exact at any size; costs one identity_route call per vertex."""
    n = int(g.n)
    vs = range(n) if vertices is None else [int(v) for v in vertices]
    full = identity_route(g)
    rows = []
    for v in vs:
        sub = identity_route(delete_vertex(g, v))
        rows.append([a - b for a, b in zip(full, sub)])
    return np.array(rows, dtype=np.uint64).reshape(len(rows), 17)


LOCAL_NAMES = ["T", "S", "I", "TT1", "TT0", "TS1", "TS0", "TI1", "SS1", "SuSv1", "SS0",
               "SuSv0", "SI1", "TI0", "SI0", "II1", "II0"]
# graphlet (index into the 17-vector) of each local term, and how many edges
# that graphlet has (each copy is seen from every one of its edges)
LOCAL_GRAPHLET = [2, 3, 4, 6, 7, 7, 8, 8, 8, 9, 10, 11, 11, 12, 13, 14, 15]
GRAPHLET_EDGES = {2: 3, 3: 2, 4: 1, 6: 6, 7: 5, 8: 4, 9: 4, 10: 3, 11: 3, 12: 3, 13: 2, 14: 2,
                  15: 1}


def _local(fn, g, eu, ev) -> np.ndarray:
    n, rp, col = _csr(g)
    eu = np.ascontiguousarray(eu, dtype=np.int32)
    ev = np.ascontiguousarray(ev, dtype=np.int32)
    k = eu.shape[0]
    out = np.zeros((max(k, 1), 17), dtype=np.int64)
    if k:
        rc = fn(n, rp.ctypes.data, col.ctypes.data, k, eu.ctypes.data, ev.ctypes.data,
                out.ctypes.data)
        if rc != 0:
            raise ValueError(f"edge-local oracle failed (code {rc})")
    return out[:k]


def edge_local(g, eu, ev) -> np.ndarray:
    """[k, 17] per-edge local vectors (LOCAL_NAMES) by vertex types, Section 4.2."""
    return _local(_load().oracle_edge_local, g, eu, ev)


def edge_local_brute(g, eu, ev) -> np.ndarray:
    """The same vectors by classifying every 3- and 4-subset containing the edge."""
    return _local(_load().oracle_edge_local_brute, g, eu, ev)


def per_edge(g, eu, ev) -> tuple[np.ndarray, np.ndarray, np.ndarray]:
    """(|Tri_e|, 4-cliques through e, induced 4-cycles through e) for each listed edge."""
    n, rp, col = _csr(g)
    eu = np.ascontiguousarray(eu, dtype=np.int32)
    ev = np.ascontiguousarray(ev, dtype=np.int32)
    k = eu.shape[0]
    T = np.zeros(max(k, 1), dtype=np.int64)
    K4 = np.zeros(max(k, 1), dtype=np.int64)
    C4 = np.zeros(max(k, 1), dtype=np.int64)
    if k:
        rc = _load().oracle_per_edge(n, rp.ctypes.data, col.ctypes.data, k, eu.ctypes.data,
                                     ev.ctypes.data, T.ctypes.data, K4.ctypes.data,
                                     C4.ctypes.data)
        if rc != 0:
            raise ValueError(f"oracle_per_edge failed (code {rc})")
    return T[:k], K4[:k], C4[:k]


def bruteforce_edge4(g, eu, ev) -> tuple[np.ndarray, np.ndarray]:
    """(4-cliques, induced 4-cycles) containing each listed edge, by subset enumeration."""
    n, rp, col = _csr(g)
    eu = np.ascontiguousarray(eu, dtype=np.int32)
    ev = np.ascontiguousarray(ev, dtype=np.int32)
    k = eu.shape[0]
    K4 = np.zeros(max(k, 1), dtype=np.int64)
    C4 = np.zeros(max(k, 1), dtype=np.int64)
    if k:
        rc = _load().oracle_bruteforce_edge4(n, rp.ctypes.data, col.ctypes.data, k,
                                             eu.ctypes.data, ev.ctypes.data, K4.ctypes.data,
                                             C4.ctypes.data)
        if rc != 0:
            raise ValueError(f"oracle_bruteforce_edge4 failed (code {rc})")
    return K4[:k], C4[:k]
