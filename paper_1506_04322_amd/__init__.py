"""Python binding of the MI355X graphlet counting library (libgraphlet.so).

Argument marshalling only: every step of the computation runs in the HIP
kernels of libgraphlet.so.  PyTorch supplies device memory and the stream.
There is no fallback: if the library is not built, or no GPU is visible, the
calls raise.

The entry points mirror include/graphlet.h:
  graphlet_count(row_ptr, col, n, per_edge=False, workspace=None, validate=False)
  graphlet_workspace_size(row_ptr, col, n, per_edge=False)
  graphlet_count_batched(node_off, row_ptr, col)
  BatchPlan(node_off, row_ptr, col, tune=True).run()   (graphlet_batch_plan_*)
  Server(budget_bytes, slots)                          (gc_server_*)
  graphlet_last_error()
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgraphlet.so")

NAMES = ["g2_1", "g2_2", "g3_1", "g3_2", "g3_3", "g3_4"] + [f"g4_{i}" for i in range(1, 12)]

GC_VALIDATE = 1
GC_DENSE_ALL = 2
GC_DENSE_OFF = 4
GC_SERVE_NO_LANE = 256
ERRORS = {
    -1: "GC_EINVAL", -2: "GC_ENOTSORTED", -3: "GC_ESELFLOOP", -4: "GC_EASYMMETRIC",
    -5: "GC_EOVERFLOW", -6: "GC_ENOMEM", -7: "GC_EHIP", -8: "GC_EINTERNAL",
}
BATCH_MAX_N = 1024
NOALLOC_MAX_GRAPHS = 65536


class GraphletError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


class _Csr(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("nnz", ctypes.c_int64),
                ("row_ptr", ctypes.c_void_p), ("col", ctypes.c_void_p)]


class _Batch(ctypes.Structure):
    _fields_ = [("graphs", ctypes.c_int64), ("node_off", ctypes.c_void_p),
                ("row_ptr", ctypes.c_void_p), ("col", ctypes.c_void_p)]


class _U128(ctypes.Structure):
    _fields_ = [("lo", ctypes.c_uint64), ("hi", ctypes.c_uint64)]


_lib = None

# Every symbol include/graphlet.h declares.
EXPORTS = [
    "graphlet_workspace_size",
    "graphlet_workspace_bound",
    "graphlet_count",
    "graphlet_count_local",
    "graphlet_count_vertex",
    "graphlet_update_edge",
    "graphlet_count_batched",
    "graphlet_count_batched_noalloc",
    "graphlet_batch_vertex",
    "graphlet_batch_gfd",
    "graphlet_batch_plan_create",
    "graphlet_batch_plan_run",
    "graphlet_batch_plan_info",
    "graphlet_batch_plan_reshape",
    "graphlet_batch_plan_destroy",
    "graphlet_last_error",
    "graphlet_version",
    "graphlet_timing_enable",
    "graphlet_last_timing",
    "gc_server_create",
    "gc_server_submit",
    "gc_server_register",
    "gc_server_update",
    "gc_server_graph_counts",
    "gc_server_unregister",
    "gc_server_poll",
    "gc_server_wait",
    "gc_server_cancel",
    "gc_server_release",
    "gc_server_stats",
    "gc_server_reset_stats",
    "gc_server_destroy",
    "gc_server_last_error",
]


class _ServeStats(ctypes.Structure):
    _fields_ = [(name, ctypes.c_int64) for name in
                ("submitted", "completed", "failed", "rejected", "cancelled", "pending",
                 "running")] + \
               [(name, ctypes.c_size_t) for name in ("bytes_in_use", "bytes_peak", "budget")] + \
               [(name, ctypes.c_double) for name in
                ("p50_ms", "p99_ms", "mean_ms", "elapsed_s", "graphs_per_s", "edges_per_s")] + \
               [(name, ctypes.c_int64) for name in ("batches", "batched")]

class _PlanInfo(ctypes.Structure):
    _fields_ = [("block", ctypes.c_int), ("classes", ctypes.c_int),
                ("class_words", ctypes.c_int * 8), ("class_graphs", ctypes.c_int64 * 8),
                ("class_grid", ctypes.c_int * 8), ("class_lds", ctypes.c_size_t * 8),
                ("candidates", ctypes.c_int), ("tuned_ms", ctypes.c_double)]


PHASES = ["prepass", "cliques", "cyc_light", "cyc_dense", "cyc_heavy", "per_edge", "step3",
          "vertex"]


class _Timing(ctypes.Structure):
    _fields_ = [("ms", ctypes.c_double * 8), ("clique_entries", ctypes.c_uint64),
                ("wedges_light", ctypes.c_uint64), ("wedges_heavy", ctypes.c_uint64),
                ("heavy_items", ctypes.c_int64), ("wedges_dense", ctypes.c_uint64),
                ("dense_hubs", ctypes.c_int64), ("clique_class", ctypes.c_int64 * 6)]


def load():
    """Loads libgraphlet.so (raises if it is missing: there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    lib.graphlet_workspace_size.argtypes = [ctypes.POINTER(_Csr), ctypes.c_int, P]
    lib.graphlet_workspace_size.restype = ctypes.c_size_t
    lib.graphlet_workspace_bound.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_int]
    lib.graphlet_workspace_bound.restype = ctypes.c_size_t
    lib.graphlet_count.argtypes = [ctypes.POINTER(_Csr), ctypes.POINTER(_U128), P, P,
                                   ctypes.c_size_t, P, ctypes.c_uint32]
    lib.graphlet_count.restype = ctypes.c_int
    lib.graphlet_count_local.argtypes = [ctypes.POINTER(_Csr), ctypes.POINTER(_U128), P, P,
                                         ctypes.c_size_t, P, ctypes.c_uint32]
    lib.graphlet_count_local.restype = ctypes.c_int
    lib.graphlet_count_vertex.argtypes = [ctypes.POINTER(_Csr), ctypes.POINTER(_U128), P, P,
                                         ctypes.c_size_t, P, ctypes.c_uint32]
    lib.graphlet_count_vertex.restype = ctypes.c_int
    lib.graphlet_update_edge.argtypes = [ctypes.POINTER(_Csr), ctypes.c_int32, ctypes.c_int32,
                                         ctypes.c_int, ctypes.POINTER(_U128), P]
    lib.graphlet_update_edge.restype = ctypes.c_int
    lib.graphlet_batch_gfd.argtypes = [P, ctypes.c_int64, P, ctypes.c_int, P]
    lib.graphlet_batch_gfd.restype = ctypes.c_int
    lib.graphlet_count_batched.argtypes = [ctypes.POINTER(_Batch), P, P, ctypes.c_uint32]
    lib.graphlet_count_batched.restype = ctypes.c_int
    lib.graphlet_count_batched_noalloc.argtypes = [ctypes.POINTER(_Batch), P, P, ctypes.c_uint32]
    lib.graphlet_count_batched_noalloc.restype = ctypes.c_int
    lib.graphlet_batch_vertex.argtypes = [ctypes.POINTER(_Batch), P, P, ctypes.c_uint32]
    lib.graphlet_batch_vertex.restype = ctypes.c_int
    lib.graphlet_batch_plan_create.argtypes = [ctypes.POINTER(_Batch), P, ctypes.c_int, P,
                                               ctypes.c_uint32, ctypes.POINTER(ctypes.c_void_p)]
    lib.graphlet_batch_plan_create.restype = ctypes.c_int
    lib.graphlet_batch_plan_run.argtypes = [P, P]
    lib.graphlet_batch_plan_run.restype = ctypes.c_int
    lib.graphlet_batch_plan_info.argtypes = [P, ctypes.POINTER(_PlanInfo)]
    lib.graphlet_batch_plan_info.restype = ctypes.c_int
    lib.graphlet_batch_plan_reshape.argtypes = [P, ctypes.c_int, ctypes.c_uint32, P]
    lib.graphlet_batch_plan_reshape.restype = ctypes.c_int
    lib.graphlet_batch_plan_destroy.argtypes = [P]
    lib.graphlet_batch_plan_destroy.restype = None
    lib.graphlet_last_error.argtypes = []
    lib.graphlet_last_error.restype = ctypes.c_char_p
    lib.graphlet_version.argtypes = []
    lib.graphlet_version.restype = ctypes.c_char_p
    lib.graphlet_timing_enable.argtypes = [ctypes.c_int]
    lib.graphlet_timing_enable.restype = None
    lib.graphlet_last_timing.argtypes = [ctypes.POINTER(_Timing)]
    lib.graphlet_last_timing.restype = ctypes.c_int
    lib.gc_server_create.argtypes = [ctypes.c_size_t, ctypes.c_int, ctypes.c_uint32]
    lib.gc_server_create.restype = ctypes.c_void_p
    lib.gc_server_submit.argtypes = [P, ctypes.c_int64, ctypes.c_int64, P, P]
    lib.gc_server_submit.restype = ctypes.c_int64
    lib.gc_server_register.argtypes = [P, ctypes.c_int64, ctypes.c_int64, P, P]
    lib.gc_server_register.restype = ctypes.c_int64
    lib.gc_server_update.argtypes = [P, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32,
                                     ctypes.c_int]
    lib.gc_server_update.restype = ctypes.c_int64
    lib.gc_server_graph_counts.argtypes = [P, ctypes.c_int64, ctypes.POINTER(_U128)]
    lib.gc_server_graph_counts.restype = ctypes.c_int
    lib.gc_server_unregister.argtypes = [P, ctypes.c_int64]
    lib.gc_server_unregister.restype = ctypes.c_int
    for f in (lib.gc_server_poll, lib.gc_server_wait):
        f.argtypes = [P, ctypes.c_int64, ctypes.POINTER(_U128), ctypes.POINTER(ctypes.c_double)]
        f.restype = ctypes.c_int
    for f in (lib.gc_server_cancel, lib.gc_server_release):
        f.argtypes = [P, ctypes.c_int64]
        f.restype = ctypes.c_int
    lib.gc_server_stats.argtypes = [P, ctypes.POINTER(_ServeStats)]
    lib.gc_server_stats.restype = ctypes.c_int
    lib.gc_server_reset_stats.argtypes = [P]
    lib.gc_server_reset_stats.restype = ctypes.c_int
    lib.gc_server_destroy.argtypes = [P]
    lib.gc_server_destroy.restype = None
    lib.gc_server_last_error.argtypes = []
    lib.gc_server_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


def graphlet_last_error() -> str:
    return load().graphlet_last_error().decode()


def _stream_ptr(stream=None) -> int:
    import torch

    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def _check_dev(t, dtype, name):
    import torch

    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


def _csr(row_ptr, col, n):
    import torch

    _check_dev(row_ptr, torch.int32, "row_ptr")
    _check_dev(col, torch.int32, "col")
    if row_ptr.numel() != n + 1:
        raise ValueError("row_ptr must have n+1 entries")
    return _Csr(int(n), int(col.numel()), row_ptr.data_ptr(), col.data_ptr() if col.numel() else 0)


def graphlet_workspace_size(row_ptr, col, n: int, per_edge=False, stream=None) -> int:
    lib = load()
    g = _csr(row_ptr, col, n)
    size = lib.graphlet_workspace_size(ctypes.byref(g), int(per_edge), _stream_ptr(stream))
    if size == 0:
        raise GraphletError(-1, graphlet_last_error())
    return int(size)


def graphlet_workspace_bound(n: int, nnz: int, per_edge=False) -> int:
    """Workspace bytes that suffice for any graph of n vertices and nnz
    adjacency entries (host arithmetic only; per_edge: False/True or 0/1/2)."""
    size = load().graphlet_workspace_bound(int(n), int(nnz), int(per_edge))
    if size == 0:
        raise GraphletError(-1, graphlet_last_error())
    return size


def graphlet_count(row_ptr, col, n: int, per_edge: bool = False, workspace=None,
                   validate: bool = False, stream=None, per_edge_out=None, dense: str = "auto"):
    """17 exact counts (python ints) of one graph; with per_edge, also a
    device int64 tensor [3, m] (|Tri_e|, 4-cliques, induced 4-cycles per
    canonical edge).  `dense` picks the route of the costliest 4-cycle
    vertices: "auto" (cost model), "all" (GC_DENSE_ALL) or "off"."""
    import torch

    lib = load()
    g = _csr(row_ptr, col, n)
    m = g.nnz // 2
    pe = None
    if per_edge:
        if per_edge_out is not None:
            _check_dev(per_edge_out, torch.int64, "per_edge_out")
            if per_edge_out.numel() < 3 * m:
                raise ValueError("per_edge_out too small")
            pe = per_edge_out
        else:
            pe = torch.empty((3, max(m, 1)), dtype=torch.int64, device=row_ptr.device)
    ws_ptr, ws_bytes = 0, 0
    if workspace is not None:
        _check_dev(workspace, torch.uint8, "workspace")
        ws_ptr, ws_bytes = workspace.data_ptr(), workspace.numel()
    out = (_U128 * 17)()
    flags = (GC_VALIDATE if validate else 0) | {"auto": 0, "all": GC_DENSE_ALL,
                                                  "off": GC_DENSE_OFF}[dense]
    rc = lib.graphlet_count(ctypes.byref(g), out, pe.data_ptr() if pe is not None else 0,
                            ws_ptr, ws_bytes, _stream_ptr(stream), flags)
    if rc != 0:
        raise GraphletError(rc, graphlet_last_error())
    counts = [int(o.lo) | (int(o.hi) << 64) for o in out]
    if per_edge:
        return counts, pe[:, :m] if pe.dim() == 2 else pe
    return counts


LOCAL = 17
LOCAL_NAMES = ["T", "S", "I", "TT1", "TT0", "TS1", "TS0", "TI1", "SS1", "SuSv1", "SS0",
               "SuSv0", "SI1", "TI0", "SI0", "II1", "II0"]


def graphlet_count_local(row_ptr, col, n: int, workspace=None, validate: bool = False,
                         stream=None, out=None):
    """(17 counts, device int64 tensor [17, m]): the per-edge local 4-node
    vectors (terms LOCAL_NAMES) in canonical edge order."""
    import torch

    lib = load()
    g = _csr(row_ptr, col, n)
    m = g.nnz // 2
    if out is None:
        out = torch.empty((LOCAL, max(m, 1)), dtype=torch.int64, device=row_ptr.device)
    else:
        _check_dev(out, torch.int64, "out")
        if out.numel() < LOCAL * m:
            raise ValueError("out too small")
    ws_ptr, ws_bytes = 0, 0
    if workspace is not None:
        _check_dev(workspace, torch.uint8, "workspace")
        ws_ptr, ws_bytes = workspace.data_ptr(), workspace.numel()
    res = (_U128 * 17)()
    rc = lib.graphlet_count_local(ctypes.byref(g), res, out.data_ptr(), ws_ptr, ws_bytes,
                                  _stream_ptr(stream), GC_VALIDATE if validate else 0)
    if rc != 0:
        raise GraphletError(rc, graphlet_last_error())
    counts = [int(o.lo) | (int(o.hi) << 64) for o in res]
    return counts, out.view(-1)[:LOCAL * m].view(LOCAL, m)


def graphlet_count_vertex(row_ptr, col, n: int, workspace=None, validate: bool = False,
                          stream=None, out=None):
    """(17 counts, device uint64 tensor [17, n]): for each vertex, the number of
    k-subsets containing it by induced class (order of NAMES)."""
    import torch

    lib = load()
    g = _csr(row_ptr, col, n)
    if out is None:
        out = torch.empty((17, max(n, 1)), dtype=torch.uint64, device=row_ptr.device)
    else:
        _check_dev(out, torch.uint64, "out")
        if out.numel() < 17 * n:
            raise ValueError("out too small")
    ws_ptr, ws_bytes = 0, 0
    if workspace is not None:
        _check_dev(workspace, torch.uint8, "workspace")
        ws_ptr, ws_bytes = workspace.data_ptr(), workspace.numel()
    res = (_U128 * 17)()
    rc = lib.graphlet_count_vertex(ctypes.byref(g), res, out.data_ptr(), ws_ptr, ws_bytes,
                                   _stream_ptr(stream), GC_VALIDATE if validate else 0)
    if rc != 0:
        raise GraphletError(rc, graphlet_last_error())
    counts = [int(o.lo) | (int(o.hi) << 64) for o in res]
    return counts, out.view(-1)[:17 * n].view(17, n)


def graphlet_update_edge(row_ptr, col, n: int, u: int, v: int, insert: bool, counts,
                         stream=None) -> list:
    """The 17 counts after inserting (or removing) the edge (u, v) of the
    graph given by (row_ptr, col), whose counts are `counts`."""
    lib = load()
    g = _csr(row_ptr, col, n)
    arr = (_U128 * 17)()
    for i, c in enumerate(counts):
        arr[i].lo = int(c) & ((1 << 64) - 1)
        arr[i].hi = int(c) >> 64
    rc = lib.graphlet_update_edge(ctypes.byref(g), int(u), int(v), 1 if insert else 0, arr,
                                  _stream_ptr(stream))
    if rc != 0:
        raise GraphletError(rc, graphlet_last_error())
    return [int(o.lo) | (int(o.hi) << 64) for o in arr]


def graphlet_count_batched(node_off, row_ptr, col, out=None, stream=None, validate=False):
    """[G, 17] int64 device tensor of the counts of every graph of a batch."""
    import torch

    lib = load()
    _check_dev(node_off, torch.int64, "node_off")
    _check_dev(row_ptr, torch.int32, "row_ptr")
    _check_dev(col, torch.int32, "col")
    G = node_off.numel() - 1
    if out is None:
        out = torch.empty((max(G, 1), 17), dtype=torch.int64, device=node_off.device)
    b = _Batch(G, node_off.data_ptr(), row_ptr.data_ptr(), col.data_ptr() if col.numel() else 0)
    rc = lib.graphlet_count_batched(ctypes.byref(b), out.data_ptr(), _stream_ptr(stream),
                                    GC_VALIDATE if validate else 0)
    if rc != 0:
        raise GraphletError(rc, graphlet_last_error())
    return out[:G]


def graphlet_count_batched_noalloc(node_off, row_ptr, col, out, stream=None, validate=False):
    """graphlet_count_batched into the caller's [G, 17] int64 device tensor
    `out`, through the entry point that allocates no device memory (at most
    NOALLOC_MAX_GRAPHS graphs)."""
    import torch

    lib = load()
    _check_dev(node_off, torch.int64, "node_off")
    _check_dev(row_ptr, torch.int32, "row_ptr")
    _check_dev(col, torch.int32, "col")
    _check_dev(out, torch.int64, "out")
    G = node_off.numel() - 1
    if out.numel() < 17 * G:
        raise ValueError("out too small")
    b = _Batch(G, node_off.data_ptr(), row_ptr.data_ptr(), col.data_ptr() if col.numel() else 0)
    rc = lib.graphlet_count_batched_noalloc(ctypes.byref(b), out.data_ptr(), _stream_ptr(stream),
                                            GC_VALIDATE if validate else 0)
    if rc != 0:
        raise GraphletError(rc, graphlet_last_error())
    return out.view(-1)[:17 * G].view(G, 17)


def graphlet_batch_vertex(node_off, row_ptr, col, out=None, stream=None, validate=False):
    """[node_off[G], 17] uint64 device tensor: for every vertex of every graph
    of a batch, the number of k-subsets of its graph containing it by induced
    class (order of NAMES); row node_off[g] + i is vertex i of graph g."""
    import torch

    lib = load()
    _check_dev(node_off, torch.int64, "node_off")
    _check_dev(row_ptr, torch.int32, "row_ptr")
    _check_dev(col, torch.int32, "col")
    G = node_off.numel() - 1
    nv = int(node_off[-1].item()) if G > 0 else 0
    if out is None:
        out = torch.empty((max(nv, 1), 17), dtype=torch.uint64, device=node_off.device)
    else:
        _check_dev(out, torch.uint64, "out")
        if out.numel() < 17 * nv:
            raise ValueError("out too small")
    b = _Batch(G, node_off.data_ptr(), row_ptr.data_ptr(), col.data_ptr() if col.numel() else 0)
    rc = lib.graphlet_batch_vertex(ctypes.byref(b), out.data_ptr(), _stream_ptr(stream),
                                   GC_VALIDATE if validate else 0)
    if rc != 0:
        raise GraphletError(rc, graphlet_last_error())
    return out.view(-1)[:17 * nv].view(nv, 17)


def graphlet_batch_gfd(counts, connected_only: bool = False, stream=None):
    """[G, 17] float64 device tensor: per size k, each count over the sum of
    the size-k counts (all classes, or the connected ones only)."""
    import torch

    lib = load()
    _check_dev(counts, torch.int64, "counts")
    counts = counts.contiguous()
    G = counts.shape[0]
    out = torch.empty((max(G, 1), 17), dtype=torch.float64, device=counts.device)
    rc = lib.graphlet_batch_gfd(counts.data_ptr(), G, out.data_ptr(), 1 if connected_only else 0,
                                _stream_ptr(stream))
    if rc != 0:
        raise GraphletError(rc, graphlet_last_error())
    return out[:G]


class BatchPlan:
    """A batch counted repeatedly: cost-ordered bins, a persistent launch
    captured in a HIP graph, optionally autotuned (graphlet_batch_plan_*).
    The tensors must stay alive and keep their sizes while the plan lives."""

    def __init__(self, node_off, row_ptr, col, tune: bool = True, out=None, stream=None,
                 validate: bool = False):
        import torch

        lib = load()
        _check_dev(node_off, torch.int64, "node_off")
        _check_dev(row_ptr, torch.int32, "row_ptr")
        _check_dev(col, torch.int32, "col")
        self.G = node_off.numel() - 1
        if out is None:
            out = torch.empty((max(self.G, 1), 17), dtype=torch.int64, device=node_off.device)
        self._keep = (node_off, row_ptr, col, out)
        self.out = out
        b = _Batch(self.G, node_off.data_ptr(), row_ptr.data_ptr(),
                   col.data_ptr() if col.numel() else 0)
        h = ctypes.c_void_p()
        rc = lib.graphlet_batch_plan_create(ctypes.byref(b), out.data_ptr(), 1 if tune else 0,
                                            _stream_ptr(stream), GC_VALIDATE if validate else 0,
                                            ctypes.byref(h))
        if rc != 0:
            raise GraphletError(rc, graphlet_last_error())
        self._h = h.value

    def run(self, stream=None):
        """Replays the captured launch; returns the [G, 17] int64 counts."""
        rc = load().graphlet_batch_plan_run(self._h, _stream_ptr(stream))
        if rc != 0:
            raise GraphletError(rc, graphlet_last_error())
        return self.out[:self.G]

    def reshape(self, block: int, class_words, stream=None) -> None:
        """Forces a workgroup size and the size classes (words per row)."""
        mask = 0
        for w in class_words:
            mask |= 1 << (int(w) - 1)
        rc = load().graphlet_batch_plan_reshape(self._h, block, mask, _stream_ptr(stream))
        if rc != 0:
            raise GraphletError(rc, graphlet_last_error())

    def info(self) -> dict:
        i = _PlanInfo()
        rc = load().graphlet_batch_plan_info(self._h, ctypes.byref(i))
        if rc != 0:
            raise GraphletError(rc, graphlet_last_error())
        k = i.classes
        return {"block": i.block, "classes": k, "class_words": list(i.class_words[:k]),
                "class_graphs": list(i.class_graphs[:k]), "class_grid": list(i.class_grid[:k]),
                "class_lds": list(i.class_lds[:k]), "candidates": i.candidates,
                "tuned_ms": i.tuned_ms}

    def close(self):
        if getattr(self, "_h", None):
            load().graphlet_batch_plan_destroy(self._h)
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def graphlet_timing_enable(on: bool = True) -> None:
    """Record per-phase device times of this thread's graphlet_count calls."""
    load().graphlet_timing_enable(1 if on else 0)


def graphlet_last_timing() -> dict:
    """Phase times (ms) and work counters of this thread's last graphlet_count."""
    t = _Timing()
    load().graphlet_last_timing(ctypes.byref(t))
    d = {f"{p}_ms": float(t.ms[i]) for i, p in enumerate(PHASES)}
    d.update(clique_entries=int(t.clique_entries), wedges_light=int(t.wedges_light),
             wedges_heavy=int(t.wedges_heavy), heavy_items=int(t.heavy_items),
             wedges_dense=int(t.wedges_dense), dense_hubs=int(t.dense_hubs),
             clique_class=[int(x) for x in t.clique_class])
    return d


class Server:
    """Continuous-batching server over the C ABI (gc_server_*).

    submit() takes host numpy CSR arrays and returns a request id; wait() /
    poll() return the 17 counts (python ints) and the latency in ms.
    """

    def __init__(self, budget_bytes: int, slots: int = 4, validate: bool = False,
                 batch_lane: bool = True):
        self._lib = load()
        flags = (GC_VALIDATE if validate else 0) | (0 if batch_lane else GC_SERVE_NO_LANE)
        h = self._lib.gc_server_create(int(budget_bytes), int(slots), flags)
        if not h:
            raise GraphletError(-1, self._lib.gc_server_last_error().decode())
        self._h = h

    def submit(self, n: int, row_ptr, col) -> int:
        import numpy as np

        rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
        c = np.ascontiguousarray(col, dtype=np.int32)
        rid = self._lib.gc_server_submit(self._h, int(n), int(c.shape[0]), rp.ctypes.data,
                                         c.ctypes.data if c.shape[0] else None)
        if rid < 0:
            raise GraphletError(int(rid), self._lib.gc_server_last_error().decode())
        return int(rid)

    def register(self, n: int, row_ptr, col) -> int:
        """Keeps the graph resident for edge updates; returns its id (also a
        request id: wait() on it gives the initial counts)."""
        import numpy as np

        rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
        c = np.ascontiguousarray(col, dtype=np.int32)
        gid = self._lib.gc_server_register(self._h, int(n), int(c.shape[0]), rp.ctypes.data,
                                           c.ctypes.data if c.shape[0] else None)
        if gid < 0:
            raise GraphletError(int(gid), self._lib.gc_server_last_error().decode())
        return int(gid)

    def update(self, graph: int, u: int, v: int, insert: bool) -> int:
        """Queues an edge insertion or deletion on a registered graph; the
        request's result is the graph's counts after it."""
        rid = self._lib.gc_server_update(self._h, int(graph), int(u), int(v), 1 if insert else 0)
        if rid < 0:
            raise GraphletError(int(rid), self._lib.gc_server_last_error().decode())
        return int(rid)

    def graph_counts(self, graph: int):
        """Current counts of a registered graph, or None before its
        registration has been counted."""
        out = (_U128 * 17)()
        rc = self._lib.gc_server_graph_counts(self._h, int(graph), out)
        if rc < 0:
            raise GraphletError(rc, self._lib.gc_server_last_error().decode())
        if rc == 0:
            return None
        return [int(o.lo) | (int(o.hi) << 64) for o in out]

    def unregister(self, graph: int) -> None:
        rc = self._lib.gc_server_unregister(self._h, int(graph))
        if rc < 0:
            raise GraphletError(rc, self._lib.gc_server_last_error().decode())

    def _result(self, fn, rid):
        out = (_U128 * 17)()
        lat = ctypes.c_double(0.0)
        rc = fn(self._h, int(rid), out, ctypes.byref(lat))
        if rc < 0:
            raise GraphletError(rc, self._lib.gc_server_last_error().decode())
        if rc == 0:
            return None
        return [int(o.lo) | (int(o.hi) << 64) for o in out], float(lat.value)

    def poll(self, rid: int):
        """(counts, latency_ms) if finished, None if not; raises if it failed."""
        return self._result(self._lib.gc_server_poll, rid)

    def wait(self, rid: int):
        """(counts, latency_ms) once the request ends; raises if it failed."""
        return self._result(self._lib.gc_server_wait, rid)

    def cancel(self, rid: int) -> None:
        self._lib.gc_server_cancel(self._h, int(rid))

    def release(self, rid: int) -> None:
        self._lib.gc_server_release(self._h, int(rid))

    def stats(self) -> dict:
        st = _ServeStats()
        self._lib.gc_server_stats(self._h, ctypes.byref(st))
        return {name: getattr(st, name) for name, _ in _ServeStats._fields_}

    def reset_stats(self) -> None:
        self._lib.gc_server_reset_stats(self._h)

    def close(self) -> None:
        if getattr(self, "_h", None):
            self._lib.gc_server_destroy(self._h)
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
