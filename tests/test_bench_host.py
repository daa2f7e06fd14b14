"""Host logic of bench.py, no GPU: the one-GPU refusal, the check that ties a
committed traffic profile to the sources it was taken on, the roofline
arithmetic and the batched kernel's work count."""
import hashlib
import os
import subprocess
import sys
import types

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_traffic_is_read_only_for_the_sources_it_was_taken_on(tmp_path, monkeypatch):
    for rel in bench.TRAFFIC_SOURCES:
        p = tmp_path / rel
        p.parent.mkdir(parents=True, exist_ok=True)
        p.write_text(f"// {rel}\n")
    h = hashlib.sha256()
    for rel in bench.TRAFFIC_SOURCES:
        h.update((tmp_path / rel).read_bytes())
    prof = tmp_path / "profiles" / bench.TRAFFIC_PROFILES["rmat22"]
    prof.parent.mkdir()
    prof.write_text("# title: not a field\n\n"
                    "kernel: k_c4_heavy_bal\n"
                    f"source_sha256: {h.hexdigest()}\n"
                    "traffic_bytes_per_launch: 123.5\n"
                    "| table: not a field |\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.measured_traffic("k_c4_heavy_bal", "rmat22") == 123.5
    # another kernel, a field the profile lacks, a workload without a profile
    assert bench.measured_traffic("k_c4_heavy_bal<true>", "rmat22") is None
    assert bench.measured_traffic("k_c4_heavy_bal", "rmat22", "l2_hit_rate") is None
    assert bench.measured_traffic("k_c4_heavy_bal", "cl") is None
    # any edit of the sources since the counters were taken voids them
    (tmp_path / bench.TRAFFIC_SOURCES[-1]).write_text("// edited\n")
    assert bench.measured_traffic("k_c4_heavy_bal", "rmat22") is None


def test_roofline_is_algorithmic_bytes_over_kernel_time():
    _, r = bench.roofline_from_timing({"cyc_heavy_ms": 2.0, "wedges_heavy": 1e9})
    assert r["bytes_per_launch"] == 4e9  # 4 B per wedge
    assert r["achieved"] == pytest.approx(2000.0)  # GB/s
    assert r["frac"] == pytest.approx(0.25)
    assert (r["bound"], r["unit"], r["peak"], r["kernel"]) == ("hbm", "GB/s", 8000.0,
                                                              "k_c4_heavy_bal")
    _, r = bench.roofline_from_timing({"cyc_heavy_ms": 2.0, "wedges_heavy": 1e9}, per_edge=True)
    assert r["kernel"] == "k_c4_heavy_bal<true>"


def test_alu_peak_is_the_published_fp32_vector_rate_per_lane_operation():
    # 157.3 TFLOP/s counts two operations per FMA and two packed fp32 lanes
    assert 4 * bench.ALU_PEAK_TOPS == pytest.approx(157.3, rel=1e-3)


def _batch(graphs):
    """A batch in the batched call's layout from (n, edge list) pairs."""
    node_off, row_ptr, cols = [0], [0], []
    for n, edges in graphs:
        adj = [[] for _ in range(n)]
        for u, v in edges:
            adj[u].append(v)
            adj[v].append(u)
        for a in adj:
            cols += sorted(a)
            row_ptr.append(len(cols))
        node_off.append(node_off[-1] + n)
    return types.SimpleNamespace(graphs=len(graphs), node_off=np.array(node_off, np.int64),
                                 row_ptr=np.array(row_ptr, np.int64),
                                 col=np.array(cols, np.int32))


def test_batched_work_on_complete_graphs_and_additivity():
    # K_n takes the dense 4-cycle pass: one word per row (n <= 64) for each
    # edge, each triangle and each vertex pair
    def complete(n):
        return n, [(u, v) for u in range(n) for v in range(u + 1, n)]

    def c(n, k):
        from math import comb
        return comb(n, k)

    for n in (4, 5, 9, 64):
        assert bench.batch_alu_work(_batch([complete(n)]), [c(n, 3)]) == 2 * c(n, 2) + c(n, 3)
    # 65 vertices need two words per row
    assert bench.batch_alu_work(_batch([complete(65)]), [c(65, 3)]) == 2 * (2 * c(65, 2) + c(65, 3))
    # a batch's work is the sum of its graphs' work, sparse ones included
    path = (100, [(i, i + 1) for i in range(99)])
    parts = [complete(7), path, complete(5)]
    tri = [c(7, 3), 0, c(5, 3)]
    whole = bench.batch_alu_work(_batch(parts), tri)
    assert whole == sum(bench.batch_alu_work(_batch([p]), [t]) for p, t in zip(parts, tri))
    # the sparse choice still does at least a word per row for each edge
    assert bench.batch_alu_work(_batch([path]), [0]) >= 2 * 99
