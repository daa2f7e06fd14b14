"""The C-ABI library loads without a GPU and exports every declared symbol."""
import ctypes
import os
import re

import pytest

import paper_1506_04322_amd as gl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    with open(os.path.join(ROOT, "include", "graphlet.h")) as f:
        text = f.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b((?:graphlet|gc_server)_\w+)\s*\(", text)))


def test_header_declares_the_binding_exports():
    assert declared_functions() == sorted(gl.EXPORTS)


def test_library_exports_every_declared_symbol():
    if not os.path.exists(gl.LIB_PATH):
        pytest.skip("library not built")
    lib = ctypes.CDLL(gl.LIB_PATH)
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_version_and_error_without_gpu():
    if not os.path.exists(gl.LIB_PATH):
        pytest.skip("library not built")
    lib = gl.load()
    assert lib.graphlet_version().startswith(b"graphlet-mi355x")
    assert gl.graphlet_last_error() == ""


def test_null_arguments_are_rejected_without_touching_a_device():
    if not os.path.exists(gl.LIB_PATH):
        pytest.skip("library not built")
    lib = gl.load()
    assert lib.graphlet_count(None, None, None, None, 0, None, 0) == -1
    assert "null" in gl.graphlet_last_error()
    assert lib.graphlet_workspace_size(None, 0, None) == 0
    bad = gl._Csr(5, 3, 0, 0)  # odd nnz
    assert lib.graphlet_count(ctypes.byref(bad), (gl._U128 * 17)(), None, None, 0, None, 0) == -1
    # entries with no vertices: refused from the sizes (pointers never read)
    bad = gl._Csr(0, 2, 0x1000, 0x1000)
    assert lib.graphlet_count(ctypes.byref(bad), (gl._U128 * 17)(), None, None, 0, None, 0) == -1
    assert "invalid sizes" in gl.graphlet_last_error()
    assert lib.graphlet_count_batched(None, None, None, 0) == -1
    assert lib.graphlet_batch_vertex(None, None, None, 0) == -1
    assert lib.graphlet_count_vertex(None, (gl._U128 * 17)(), None, None, 0, None, 0) == -1
    assert "null" in gl.graphlet_last_error()


def test_vertex_counts_reject_large_n_before_any_device_work():
    # C(n-1, 3) >= 2^64: refused on the host from n alone (the pointers are
    # never dereferenced)
    if not os.path.exists(gl.LIB_PATH):
        pytest.skip("library not built")
    lib = gl.load()
    g = gl._Csr(4_900_000, 0, 0x1000, 0)
    rc = lib.graphlet_count_vertex(ctypes.byref(g), (gl._U128 * 17)(), 0x1000, None, 0, None, 0)
    assert rc == -5 and "64 bits" in gl.graphlet_last_error()


def test_noalloc_batched_refuses_oversized_batches_before_any_device_work():
    # the pointers are never dereferenced: the graph count alone decides
    if not os.path.exists(gl.LIB_PATH):
        pytest.skip("library not built")
    lib = gl.load()
    assert lib.graphlet_count_batched_noalloc(None, None, None, 0) == -1
    b = gl._Batch(gl.NOALLOC_MAX_GRAPHS + 1, 0x1000, 0x1000, 0)
    assert lib.graphlet_count_batched_noalloc(ctypes.byref(b), 0x1000, None, 0) == -1
    assert "allocation-free limit" in gl.graphlet_last_error()


def test_host_only_workspace_bound():
    # sizes alone: no device work, so it runs without a GPU
    if not os.path.exists(gl.LIB_PATH):
        pytest.skip("library not built")
    lib = gl.load()
    assert lib.graphlet_workspace_bound(0, 0, 0) == 256
    b0 = gl.graphlet_workspace_bound(1000, 16000, 0)
    b1 = gl.graphlet_workspace_bound(1000, 16000, 1)
    b2 = gl.graphlet_workspace_bound(1000, 16000, 2)
    assert 0 < b0 < b1 < b2
    assert gl.graphlet_workspace_bound(2000, 16000, 0) > b0
    assert gl.graphlet_workspace_bound(1000, 32000, 0) > b0
    for n, nnz, pe in ((1000, 15999, 0), (-1, 10, 0), (10, -2, 0), (10, 10, 3), (2**31, 10, 0)):
        assert lib.graphlet_workspace_bound(n, nnz, pe) == 0, (n, nnz, pe)
        assert "invalid" in gl.graphlet_last_error()


def test_binding_fails_loudly_when_library_is_missing(tmp_path, monkeypatch):
    monkeypatch.setattr(gl, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(gl, "_lib", None)
    with pytest.raises(RuntimeError):
        gl.load()
