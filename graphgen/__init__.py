"""Seeded synthetic graph inputs (host side, numpy CSR).

Inputs only: nothing here counts graphlets.  The CPU oracle and the GPU path
both take their graphs from this module.  The paper's own datasets are real
networks (Section 5); the workloads below are synthetic stand-ins with the
shapes the experiments call for (power-law, R-MAT, dense small graphs).
"""
from __future__ import annotations

import ctypes
import hashlib
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gen.cpp")
_LIB = os.path.join(_HERE, "libgraphgen.so")
_lib = None


def build() -> str:
    """Compile the generator library in place (g++, -O2)."""
    cmd = ["g++", "-O2", "-std=c++17", "-fPIC", "-shared", "-o", _LIB + ".tmp", _SRC]
    subprocess.run(cmd, check=True)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        lib.gg_make.restype = ctypes.c_void_p
        lib.gg_make.argtypes = [ctypes.c_int, ctypes.POINTER(ctypes.c_double), ctypes.c_uint64]
        for f in (lib.gg_n, lib.gg_nnz, lib.gg_graphs):
            f.restype = ctypes.c_int64
            f.argtypes = [ctypes.c_void_p]
        lib.gg_export.restype = None
        lib.gg_export.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
        lib.gg_export_batch.restype = None
        lib.gg_export_batch.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
        lib.gg_free.restype = None
        lib.gg_free.argtypes = [ctypes.c_void_p]
        _lib = lib
    return _lib


@dataclass
class Csr:
    """Undirected simple graph: row_ptr int32[n+1], col int32[2m], lists strictly increasing."""

    n: int
    row_ptr: np.ndarray
    col: np.ndarray

    @property
    def nnz(self) -> int:
        return int(self.col.shape[0])

    @property
    def m(self) -> int:
        return self.nnz // 2

    def degrees(self) -> np.ndarray:
        return np.diff(self.row_ptr.astype(np.int64))

    def sha256(self) -> str:
        h = hashlib.sha256()
        h.update(np.int64(self.n).tobytes())
        h.update(np.ascontiguousarray(self.row_ptr, dtype=np.int32).tobytes())
        h.update(np.ascontiguousarray(self.col, dtype=np.int32).tobytes())
        return h.hexdigest()


@dataclass
class Batch:
    """Many graphs in one CSR: rows concatenated, column ids local to each graph.

    node_off int64[G+1] gives each graph's row range; row_ptr indexes the
    concatenated col array.
    """

    node_off: np.ndarray
    kind: np.ndarray
    row_ptr: np.ndarray
    col: np.ndarray

    @property
    def graphs(self) -> int:
        return int(self.node_off.shape[0] - 1)

    def graph(self, i: int) -> Csr:
        a, b = int(self.node_off[i]), int(self.node_off[i + 1])
        rp = self.row_ptr[a : b + 1].astype(np.int64)
        col = self.col[rp[0] : rp[-1]].copy()
        return Csr(b - a, (rp - rp[0]).astype(np.int32), col)

    def sha256(self) -> str:
        h = hashlib.sha256()
        for arr in (self.node_off, self.row_ptr, self.col):
            h.update(np.ascontiguousarray(arr).tobytes())
        return h.hexdigest()


def _make(kind: int, params, seed: int):
    lib = _load()
    p = (ctypes.c_double * len(params))(*[float(x) for x in params])
    h = lib.gg_make(kind, p, ctypes.c_uint64(seed & 0xFFFFFFFFFFFFFFFF))
    if not h:
        raise ValueError(f"graph generator rejected kind={kind} params={params}")
    try:
        n = lib.gg_n(h)
        nnz = lib.gg_nnz(h)
        row_ptr = np.empty(n + 1, dtype=np.int32)
        col = np.empty(max(nnz, 0), dtype=np.int32)
        lib.gg_export(h, row_ptr.ctypes.data, col.ctypes.data)
        if kind == 5:
            G = lib.gg_graphs(h)
            node_off = np.empty(G + 1, dtype=np.int64)
            kinds = np.empty(G, dtype=np.int64)
            lib.gg_export_batch(h, node_off.ctypes.data, kinds.ctypes.data)
            return Batch(node_off, kinds, row_ptr, col)
        return Csr(int(n), row_ptr, col)
    finally:
        lib.gg_free(h)


def er_gnm(n: int, m: int, seed: int) -> Csr:
    """Erdos-Renyi G(n, m): m distinct uniform pairs."""
    return _make(1, [n, m], seed)


def chung_lu(n: int, beta: float, i0: float, balls: int, seed: int) -> Csr:
    """Chung-Lu power law by ball dropping, weights (i + i0)^(-1/(beta-1))."""
    return _make(2, [n, beta, i0, balls], seed)


def rmat(scale: int, edge_factor: int, a: float, b: float, c: float, seed: int) -> Csr:
    """R-MAT without noise, randomly permuted ids, symmetrised and deduplicated."""
    return _make(3, [scale, edge_factor, a, b, c], seed)


def rgg_torus(n: int, mean_degree: float, seed: int) -> Csr:
    """Random geometric graph on the unit torus with the given expected mean degree."""
    return _make(4, [n, mean_degree], seed)


def batch(G: int, nmin: int, nmax: int, rho_min: float, rho_max: float, rgg_frac: float,
          rgg_deg: float, seed: int) -> Batch:
    """G small graphs: ER G(n, rho C(n,2)) or, with probability rgg_frac, a torus RGG."""
    return _make(5, [G, nmin, nmax, rho_min, rho_max, rgg_frac, rgg_deg], seed)


def from_edges(n: int, edges) -> Csr:
    """CSR from an iterable of (u, v) pairs; loops dropped, duplicates merged."""
    e = np.asarray(list(edges), dtype=np.int64).reshape(-1, 2)
    if e.size:
        e = e[e[:, 0] != e[:, 1]]
        if e.size and (e.min() < 0 or e.max() >= n):
            raise ValueError("vertex id out of range")
        lo = np.minimum(e[:, 0], e[:, 1])
        hi = np.maximum(e[:, 0], e[:, 1])
        key = np.unique(lo * (n + 1) + hi)
        lo, hi = key // (n + 1), key % (n + 1)
        src = np.concatenate([lo, hi])
        dst = np.concatenate([hi, lo])
        order = np.lexsort((dst, src))
        src, dst = src[order], dst[order]
    else:
        src = dst = np.zeros(0, dtype=np.int64)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(row_ptr, src + 1, 1)
    row_ptr = np.cumsum(row_ptr)
    return Csr(n, row_ptr.astype(np.int32), dst.astype(np.int32))
