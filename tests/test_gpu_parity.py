"""GPU parity: the HIP path through the C ABI against the CPU oracle.

All counts are integers, so the bar is bit-exact equality everywhere: the
17-vector (Table 1 classes) and the per-edge |Tri_e|, 4-clique and induced
4-cycle counts in canonical edge order.
"""
import hashlib
import json
import os
from math import comb

import numpy as np
import pytest

import graphgen
import graphgen.configs as C
import oracle
import paper_1506_04322_amd as gl

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


def dev(a):
    import torch

    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def gpu_counts(g, per_edge=False, validate=True):
    rp = dev(g.row_ptr)
    col = dev(g.col)
    if per_edge:
        c, pe = gl.graphlet_count(rp, col, g.n, per_edge=True, validate=validate)
        return c, pe.cpu().numpy()
    return gl.graphlet_count(rp, col, g.n, validate=validate)


def check_full(g, route=oracle.identity_route, per_edge=True):
    want = route(g)
    got = gpu_counts(g)
    assert got == want, (got, want)
    if per_edge:
        got2, pe = gpu_counts(g, per_edge=True)
        assert got2 == want
        eu, ev = oracle.edges(g)
        if len(eu):
            T, K4, C4 = oracle.per_edge(g, eu, ev)
            np.testing.assert_array_equal(pe[0], T)
            np.testing.assert_array_equal(pe[1], K4)
            np.testing.assert_array_equal(pe[2], C4)


def rand_graph(rng, n, p):
    iu = np.triu_indices(n, 1)
    mask = rng.random(len(iu[0])) < p
    return graphgen.from_edges(n, list(zip(iu[0][mask], iu[1][mask])))


# ------------------------------------------------------------ small graphs


@pytest.mark.parametrize("seed", range(6))
def test_random_small_graphs_vs_bruteforce(seed):
    rng = np.random.default_rng(1000 + seed)
    for _ in range(10):
        n = int(rng.integers(0, 40))
        g = rand_graph(rng, n, float(rng.random()))
        check_full(g, route=oracle.bruteforce)


def test_empty_and_tiny():
    for n in range(0, 6):
        g = graphgen.from_edges(n, [])
        want = oracle.bruteforce(g)
        assert gpu_counts(g) == want
    g = graphgen.from_edges(3, [(0, 1)])
    check_full(g, route=oracle.bruteforce)
    g = graphgen.from_edges(2, [(0, 1)])
    check_full(g, route=oracle.bruteforce)


def test_isolated_vertices_many():
    g = graphgen.from_edges(100000, [(0, 1), (1, 2), (2, 0), (5, 6), (99999, 3)])
    check_full(g)


def test_edge_keys_ragged_tiles():
    # the prepass keys the entries in tiles of 2048 consecutive entries: a
    # row that starts inside a tile and spans several, runs of empty rows
    # between rows, nnz an exact multiple of the tile, a lone edge at the
    # last ids, trailing isolated vertices
    rng = np.random.default_rng(77)
    n = 9000
    ids = [int(v) for v in rng.permutation(n)[:2400]]
    hub, leaves = ids[0], ids[1:2101]
    edges = [(hub, v) for v in leaves]
    edges += [(leaves[i], leaves[i + 1]) for i in range(0, 600, 2)]
    edges += list(zip(ids[2101:2250], ids[2250:2399]))
    g = graphgen.from_edges(n + 500, edges)
    assert g.nnz > 4096 and np.diff(g.row_ptr).max() > 2048
    check_full(g)
    g = graphgen.from_edges(2388, [(300 + i, 300 + (i + 1) % 2048) for i in range(2048)])
    assert g.nnz == 2 * 2048
    check_full(g)
    g = graphgen.from_edges(5000, [(4998, 4999)])
    check_full(g)


def clique_classes(g, per_edge):
    """Runs the graph with timing on; returns the vertex counts per clique
    kernel class (gc_timing.clique_class) and the results."""
    gl.graphlet_timing_enable(True)
    try:
        res = gpu_counts(g, per_edge=per_edge, validate=False)
        return gl.graphlet_last_timing()["clique_class"], res
    finally:
        gl.graphlet_timing_enable(False)


def test_complete_graphs_cover_every_clique_bin():
    # K_n: |U(u)| takes every value 0 .. n-1, so K_n runs every clique class
    # with a bound below n: k <= 64, 256, 512, 1088 in LDS; in per-edge mode
    # 896 < k <= 1088 keeps its rows in a global slot; k > 1088 runs the
    # global-memory kernel in both modes
    for n in (4, 65, 300, 700, 1000, 1100):
        edges = [(a, b) for a in range(n) for b in range(a + 1, n)]
        g = graphgen.from_edges(n, edges)
        cls, got = clique_classes(g, per_edge=False)
        want = [0] * 17
        want[0], want[2], want[6] = comb(n, 2), comb(n, 3), comb(n, 4)
        assert got == want
        cls2, (got2, pe) = clique_classes(g, per_edge=True)
        assert got2 == want and cls2 == cls
        assert (pe[0] == n - 2).all() and (pe[1] == comb(n - 2, 2)).all() and (pe[2] == 0).all()
        # vertex of rank r has k = n - 1 - r upper neighbours
        ks = np.arange(n - 1, -1, -1)
        ks = ks[ks >= 2]
        assert cls[0] == int(((ks >= 2) & (ks <= 64)).sum())
        assert cls[1] == int(((ks > 64) & (ks <= 256)).sum())
        assert cls[2] == int(((ks > 256) & (ks <= 512)).sum())
        assert cls[3] == int(((ks > 512) & (ks <= 1088)).sum())
        assert cls[4] == int((ks > 1088).sum())
        assert cls[5] == int(((ks > 896) & (ks <= 1088)).sum())
    assert cls[4] > 0 and cls[5] > 0  # K_1100 ran both global-memory shapes


def hub_core_graph(na=1150, nb=1500, nc=400, pa=0.05, periphery=2000, seed=61):
    """Vertices with more than 1088 upper neighbours, at moderate clique
    counts: a set A (sparse inside, p = pa) that every vertex of C and a
    fraction q_b ~ U[0.02, 0.98] of B attach to, plus a sparse periphery.
    A has the highest degrees, so the upper neighbours of a vertex of C are
    all of A (k = 1150 > 1088) and those of b in B about q_b |A|, which
    spans every clique class, the per-edge global-slot one (896 < k <= 1088)
    included."""
    rng = np.random.default_rng(seed)
    A = np.arange(na)
    n = na + nb + nc + periphery
    iu = np.triu_indices(na, 1)
    keep = rng.random(len(iu[0])) < pa
    edges = list(zip(iu[0][keep].tolist(), iu[1][keep].tolist()))
    q = rng.uniform(0.02, 0.98, nb)
    for i in range(nb):
        b = na + i
        edges += [(int(a), b) for a in A[rng.random(na) < q[i]]]
    for i in range(nc):
        c = na + nb + i
        edges += [(int(a), c) for a in A]
    for x in range(na + nb + nc, n):
        for y in rng.integers(0, n, 3):
            if int(y) != x:
                edges.append((min(x, int(y)), max(x, int(y))))
    return graphgen.from_edges(n, edges)


def test_hub_core_every_clique_class_vs_oracle():
    g = hub_core_graph()
    want = oracle.identity_route(g)
    cls, got = clique_classes(g, per_edge=False)
    assert got == want
    cls2, (got2, pe) = clique_classes(g, per_edge=True)
    assert got2 == want
    assert all(c > 0 for c in cls), cls  # every class, both global-memory shapes
    assert int(pe[0].sum()) == 3 * want[2]
    assert int(pe[1].sum()) == 6 * want[6]
    assert int(pe[2].sum()) == 4 * want[9]
    # per-edge values against the literal per-edge oracle: edges at vertices
    # of the k > 1088 class (C), at vertices of the global-slot class
    # (b in B with 896 < k <= 1088), random edges, periphery edges
    eu, ev = oracle.edges(g)
    na, nb, nc = 1150, 1500, 400
    d = g.degrees()
    lo_end = np.maximum(eu, ev)  # the B, C or periphery end of an edge
    in_c = (lo_end >= na + nb) & (lo_end < na + nb + nc)
    in_b = (lo_end >= na) & (lo_end < na + nb)
    gslot = in_b & (d[lo_end] > 930) & (d[lo_end] < 1080)
    per = lo_end >= na + nb + nc
    rng = np.random.default_rng(62)
    idx = np.unique(np.concatenate([
        rng.choice(np.nonzero(in_c)[0], 40, replace=False),
        rng.choice(np.nonzero(gslot)[0], 40, replace=False),
        rng.choice(len(eu), 60, replace=False),
        rng.choice(np.nonzero(per)[0], 40, replace=False)]))
    T, K4, C4 = oracle.per_edge(g, eu[idx], ev[idx])
    np.testing.assert_array_equal(pe[0][idx], T)
    np.testing.assert_array_equal(pe[1][idx], K4)
    np.testing.assert_array_equal(pe[2][idx], C4)
    # local vectors through the same classes
    counts, L = gpu_local(g)
    assert counts == want
    check_local_sums(g, counts, L)
    sub = idx[rng.choice(len(idx), 60, replace=False)]
    np.testing.assert_array_equal(L[sub], oracle.edge_local(g, eu[sub], ev[sub]))


# ------------------------------------------------------------ configurations


def golden(name):
    path = os.path.join(HERE, "golden", "configs.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f).get(name)
    return d


def test_config1_er_full():
    g = C.er()
    gd = golden("er")
    assert gd is not None and gd["sha256"] == g.sha256()
    want = [int(x) for x in gd["counts"]]
    assert want == oracle.identity_route(g)
    check_full(g)


def _sampled_edges(g, k, seed):
    eu, ev = oracle.edges(g)
    rng = np.random.default_rng(seed)
    idx = np.unique(np.concatenate([rng.integers(0, len(eu), k), np.arange(min(50, len(eu)))]))
    # also the edges at the highest-degree vertex
    d = g.degrees()
    hub = int(np.argmax(d))
    hub_idx = np.nonzero((eu == hub) | (ev == hub))[0][:50]
    idx = np.unique(np.concatenate([idx, hub_idx]))
    return idx, eu[idx], ev[idx]


def test_config2_chung_lu_full_size():
    g = C.cl()
    got, pe = gpu_counts(g, per_edge=True, validate=False)
    assert got == gpu_counts(g, validate=False)
    gd = golden("cl")
    if gd is not None:
        assert gd["sha256"] == g.sha256()
        assert got == [int(x) for x in gd["counts"]]
    idx, eu, ev = _sampled_edges(g, 3000, 22)
    T, K4, C4 = oracle.per_edge(g, eu, ev)
    np.testing.assert_array_equal(pe[0][idx], T)
    np.testing.assert_array_equal(pe[1][idx], K4)
    np.testing.assert_array_equal(pe[2][idx], C4)
    # sum rules that hold at any size
    assert int(pe[0].sum()) == 3 * got[2]
    assert int(pe[1].sum()) == 6 * got[6]
    assert int(pe[2].sum()) == 4 * got[9]
    assert sum(got[2:6]) == comb(g.n, 3) and sum(got[6:]) == comb(g.n, 4)


def test_config3_rmat22_full_size():
    gd = golden("rmat")
    if gd is None:
        pytest.skip("R-MAT oracle counts not generated yet")
    g = C.rmat22()
    assert gd["sha256"] == g.sha256()
    got = gpu_counts(g, validate=False)
    assert got == [int(x) for x in gd["counts"]]
    assert got[5] > 2**63  # needs the 128-bit path


def test_config3_rmat22_per_edge_sampled():
    # per-edge mode at full size: every 4-cycle vertex takes the light, medium
    # or heavy route with credits (no dense slabs), every clique bin its
    # per-edge kernel
    gd = golden("rmat")
    if gd is None:
        pytest.skip("R-MAT oracle counts not generated yet")
    g = C.rmat22()
    got, pe = gpu_counts(g, per_edge=True, validate=False)
    assert got == [int(x) for x in gd["counts"]]
    assert int(pe[0].sum()) == 3 * got[2]
    assert int(pe[1].sum()) == 6 * got[6]
    assert int(pe[2].sum()) == 4 * got[9]
    eu, ev = oracle.edges(g)
    d = g.degrees()
    rng = np.random.default_rng(57)
    cheap = np.nonzero(d[eu] + d[ev] < 3000)[0]
    idx = rng.choice(cheap, 400, replace=False)
    # edges at the hubs (the heavy 4-cycle items, the dense-slab vertices and
    # the global-slot clique class run there) whose other end has low degree:
    # the literal oracle walks the small star side, so they stay cheap
    hubs = np.argsort(-d, kind="stable")[:40]
    lo_end = np.where(np.isin(eu, hubs), ev, eu)
    at_hub = np.nonzero((np.isin(eu, hubs) | np.isin(ev, hubs)) & (d[lo_end] <= 12))[0]
    idx = np.unique(np.concatenate([idx, rng.choice(at_hub, 120, replace=False)]))
    T, K4, C4 = oracle.per_edge(g, eu[idx], ev[idx])
    np.testing.assert_array_equal(pe[0][idx], T)
    np.testing.assert_array_equal(pe[1][idx], K4)
    np.testing.assert_array_equal(pe[2][idx], C4)


def test_dense_hub_slabs_rmat17():
    # every route of the costliest 4-cycle vertices gives the oracle's counts
    g = graphgen.rmat(17, 16, 0.57, 0.19, 0.19, 11)
    want = oracle.identity_route(g)
    rp, col = dev(g.row_ptr), dev(g.col)
    gl.graphlet_timing_enable(True)
    try:
        for route in ("all", "off", "auto"):
            assert gl.graphlet_count(rp, col, g.n, dense=route) == want, route
            t = gl.graphlet_last_timing()
            if route == "all":
                assert t["dense_hubs"] > kDenseSlab and t["wedges_dense"] > 0  # several slabs
            if route == "off":
                assert t["dense_hubs"] == 0
    finally:
        gl.graphlet_timing_enable(False)
    # the per-edge run does not use slabs and must agree
    got2, pe = gpu_counts(g, per_edge=True, validate=False)
    assert got2 == want


kDenseSlab = 256


@pytest.mark.parametrize("nv", [700, 2000, 3000, 4000])
def test_heavy_items_long_runs(nv):
    # x is adjacent to nv vertices v, each adjacent to the same 30 vertices y
    # below x in the degree order (ties by id): every list of x's heavy item
    # has a run of 30 in one chunk, longer than a thread's buffer, so all nv
    # lists go to the long-run queue together (one, two or three lists per
    # thread up to 3072 lists, groups of 2048 lists above); the y's are heavy
    # too, with runs of every length up to 29
    ny = 30
    x = ny + nv
    edges = [(y, ny + i) for i in range(nv) for y in range(ny)] + [(ny + i, x) for i in range(nv)]
    g = graphgen.from_edges(x + 1, edges)
    want = oracle.identity_route(g)
    gl.graphlet_timing_enable(True)
    try:
        got = gl.graphlet_count(dev(g.row_ptr), dev(g.col), g.n, dense="off", validate=True)
        t = gl.graphlet_last_timing()
    finally:
        gl.graphlet_timing_enable(False)
    assert got == want
    assert t["heavy_items"] >= 2 and t["wedges_heavy"] >= nv * ny
    # per-edge mode walks the same items and credits every wedge: the
    # 17-vector, the sum rules and sampled edges (x's, the y's, others)
    # against the literal per-edge oracle
    got_pe, pe = gpu_counts(g, per_edge=True, validate=False)
    assert got_pe == want
    assert int(pe[0].sum()) == 3 * want[2] and int(pe[1].sum()) == 6 * want[6]
    assert int(pe[2].sum()) == 4 * want[9]
    eu, ev = oracle.edges(g)
    rng = np.random.default_rng(nv)
    idx = np.unique(np.concatenate([rng.integers(0, len(eu), 120),
                                    np.nonzero(ev == x)[0][:40], np.nonzero(eu < ny)[0][:40]]))
    T, K4, C4 = oracle.per_edge(g, eu[idx], ev[idx])
    np.testing.assert_array_equal(pe[0][idx], T)
    np.testing.assert_array_equal(pe[1][idx], K4)
    np.testing.assert_array_equal(pe[2][idx], C4)


def hub_lists_graph(nv, ny=30):
    x = ny + nv
    edges = [(y, ny + i) for i in range(nv) for y in range(ny)] + [(ny + i, x) for i in range(nv)]
    return graphgen.from_edges(x + 1, edges)


@pytest.mark.parametrize("case", ["rmat14", "hub_lists_3000", "chung_lu_small"])
def test_per_edge_heavy_credits_packed_and_wide(case):
    # Heavy wedge credits go to 32-bit totals per entry, two neighbouring
    # entries per atomic add, unless the maximum degree exceeds 65535 (then
    # each entry takes its own 64-bit add).  A disjoint star with 65536 leaves
    # switches the graph to the wide credits and changes none of the values
    # of the original edges, which come first in canonical order.
    if case == "rmat14":
        g = graphgen.rmat(14, 16, 0.57, 0.19, 0.19, 5)
    elif case == "hub_lists_3000":
        g = hub_lists_graph(3000)
    else:
        g = graphgen.chung_lu(20000, 2.1, 13.0, 218000, 3)
    want = oracle.identity_route(g)
    gl.graphlet_timing_enable(True)
    try:
        got, pe = gpu_counts(g, per_edge=True, validate=False)
        t = gl.graphlet_last_timing()
    finally:
        gl.graphlet_timing_enable(False)
    assert got == want and t["wedges_heavy"] > 0
    assert int(pe[0].sum()) == 3 * want[2] and int(pe[1].sum()) == 6 * want[6]
    assert int(pe[2].sum()) == 4 * want[9]
    eu, ev = oracle.edges(g)
    leaves = 65536
    star = np.stack([np.full(leaves, g.n), g.n + 1 + np.arange(leaves)], axis=1)
    g2 = graphgen.from_edges(g.n + 1 + leaves, np.concatenate([np.stack([eu, ev], axis=1), star]))
    got2, pe2 = gpu_counts(g2, per_edge=True, validate=False)
    m = pe.shape[1]
    np.testing.assert_array_equal(pe2[:, :m], pe)
    assert not pe2[:, m:].any()  # a star closes no triangle or cycle
    # sampled edges, the heaviest endpoints' among them, against the literal
    # per-edge oracle
    deg = np.diff(g.row_ptr)
    rng = np.random.default_rng(7)
    top = np.argsort(deg)[-3:]
    idx = np.unique(np.concatenate([rng.integers(0, len(eu), 150)] +
                                   [np.nonzero((eu == h) | (ev == h))[0][:30] for h in top]))
    T, K4, C4 = oracle.per_edge(g, eu[idx], ev[idx])
    np.testing.assert_array_equal(pe[0][idx], T)
    np.testing.assert_array_equal(pe[1][idx], K4)
    np.testing.assert_array_equal(pe[2][idx], C4)


# ------------------------------------------------------------ per-edge local vectors


def gpu_local(g):
    counts, L = gl.graphlet_count_local(dev(g.row_ptr), dev(g.col), g.n, validate=True)
    return counts, L.cpu().numpy().T  # [m, 17]


def check_local_sums(g, counts, L):
    n = g.n
    if len(L):
        assert (L[:, :3].sum(1) == n - 2).all()
        assert (L[:, 3:].sum(1) == comb(n - 2, 2)).all()
    tot = {}
    for j, G in enumerate(oracle.LOCAL_GRAPHLET):
        tot[G] = tot.get(G, 0) + int(L[:, j].sum())
    for G, s in tot.items():
        assert s == oracle.GRAPHLET_EDGES[G] * counts[G], G


@pytest.mark.parametrize("seed", range(4))
def test_edge_local_small_graphs_vs_oracle(seed):
    rng = np.random.default_rng(3000 + seed)
    for _ in range(8):
        n = int(rng.integers(2, 60))
        g = rand_graph(rng, n, float(rng.random()))
        counts, L = gpu_local(g)
        assert counts == oracle.bruteforce(g)
        eu, ev = oracle.edges(g)
        if len(eu):
            np.testing.assert_array_equal(L, oracle.edge_local(g, eu, ev))
        check_local_sums(g, counts, L)


def test_edge_local_skewed_graphs():
    for g in (graphgen.rmat(13, 16, 0.57, 0.19, 0.19, 12),
              graphgen.chung_lu(5000, 2.1, 3.0, 60000, 8),
              graphgen.from_edges(400, [(0, i) for i in range(1, 400)] +
                                  [(1, i) for i in range(2, 400)])):
        counts, L = gpu_local(g)
        assert counts == oracle.identity_route(g)
        check_local_sums(g, counts, L)
        idx, eu, ev = _sampled_edges(g, 300, 31)
        np.testing.assert_array_equal(L[idx], oracle.edge_local(g, eu, ev))
        # the per-edge arrays of graphlet_count are the same numbers
        _, pe = gpu_counts(g, per_edge=True, validate=False)
        np.testing.assert_array_equal(pe[0], L[:, 0])
        np.testing.assert_array_equal(pe[1], L[:, 3])
        np.testing.assert_array_equal(pe[2], L[:, 9])


def test_edge_local_chung_lu_full_size():
    g = C.cl()
    counts, L = gpu_local(g)
    gd = golden("cl")
    assert gd is not None and counts == [int(x) for x in gd["counts"]]
    n = g.n
    assert (L[:, :3].sum(1) == n - 2).all()
    assert (L[:, 3:].sum(1) == comb(n - 2, 2)).all()
    for G in sorted(set(oracle.LOCAL_GRAPHLET)):
        cols = [j for j, x in enumerate(oracle.LOCAL_GRAPHLET) if x == G]
        per_edge = L[:, cols].sum(1)  # each below 2^40
        tot = sum(int(c.sum()) for c in np.array_split(per_edge, 64))  # exact
        assert tot == oracle.GRAPHLET_EDGES[G] * counts[G], G
    idx, eu, ev = _sampled_edges(g, 24, 41)
    keep = np.concatenate([idx[:20], idx[-20:]])
    sel = np.isin(idx, keep)
    np.testing.assert_array_equal(L[idx[sel]], oracle.edge_local(g, eu[sel], ev[sel]))


# ------------------------------------------------------------ per-vertex counts


def gpu_vertex(g, validate=True):
    counts, V = gl.graphlet_count_vertex(dev(g.row_ptr), dev(g.col), g.n, validate=validate)
    return counts, V.cpu().numpy().T  # [n, 17] uint64


def exact_sum(col):
    """Exact integer sum of a uint64 column (numpy sums in 32-bit halves)."""
    col = np.asarray(col, dtype=np.uint64)
    lo = int((col & np.uint64(0xFFFFFFFF)).sum(dtype=np.uint64))
    hi = int((col >> np.uint64(32)).sum(dtype=np.uint64))
    return lo + (hi << 32)


def check_vertex_sums(g, counts, V):
    for c in range(17):
        assert exact_sum(V[:, c]) == oracle.CLASS_K[c] * counts[c], oracle.NAMES[c]
    np.testing.assert_array_equal(V[:, 0], g.degrees().astype(np.uint64))
    n = g.n
    if n:
        assert (V[:, :2].sum(1) == n - 1).all()
        assert (V[:, 2:6].sum(1) == np.uint64(comb(n - 1, 2))).all()
        assert (V[:, 6:].sum(1) == np.uint64(comb(n - 1, 3))).all()


def _sampled_vertices(g, k, seed):
    rng = np.random.default_rng(seed)
    d = g.degrees()
    top = np.argsort(-d, kind="stable")[:10]
    zero = np.nonzero(d == 0)[0][:3]
    return np.unique(np.concatenate([rng.integers(0, g.n, k), top, zero, [0, g.n - 1]]))


@pytest.mark.parametrize("seed", range(4))
def test_vertex_counts_small_graphs_vs_bruteforce(seed):
    rng = np.random.default_rng(5000 + seed)
    for _ in range(8):
        n = int(rng.integers(1, 60))
        g = rand_graph(rng, n, float(rng.random()))
        counts, V = gpu_vertex(g)
        assert counts == oracle.bruteforce(g)
        np.testing.assert_array_equal(V, oracle.vertex_bruteforce(g).astype(np.uint64))


def test_vertex_counts_edge_cases():
    cases = [graphgen.from_edges(0, []), graphgen.from_edges(1, []),
             graphgen.from_edges(6, []), graphgen.from_edges(2, [(0, 1)]),
             graphgen.from_edges(300, [(0, i) for i in range(1, 300)]),
             graphgen.from_edges(40, [(a, b) for a in range(40) for b in range(a + 1, 40)]),
             graphgen.from_edges(200, [(2 * i, 2 * i + 1) for i in range(100)])]
    for g in cases:
        counts, V = gpu_vertex(g)
        assert V.shape == (g.n, 17)
        assert counts == oracle.identity_route(g)
        if g.n <= 60:
            np.testing.assert_array_equal(V, oracle.vertex_bruteforce(g).astype(np.uint64))
        else:
            vs = _sampled_vertices(g, 20, 7)
            np.testing.assert_array_equal(V[vs], oracle.vertex_by_deletion(g, vs))
        check_vertex_sums(g, counts, V)


def test_vertex_counts_config1_every_vertex_by_deletion():
    g = C.er()
    counts, V = gpu_vertex(g)
    np.testing.assert_array_equal(V, oracle.vertex_by_deletion(g))
    check_vertex_sums(g, counts, V)


def test_vertex_counts_skewed_graphs_sampled():
    for g in (graphgen.rmat(12, 16, 0.57, 0.19, 0.19, 5),
              graphgen.chung_lu(5000, 2.1, 3.0, 60000, 8),
              graphgen.from_edges(400, [(0, i) for i in range(1, 400)] +
                                  [(1, i) for i in range(2, 400)])):
        counts, V = gpu_vertex(g, validate=False)
        assert counts == oracle.identity_route(g)
        check_vertex_sums(g, counts, V)
        vs = _sampled_vertices(g, 60, 17)
        np.testing.assert_array_equal(V[vs], oracle.vertex_by_deletion(g, vs))


def test_vertex_counts_chung_lu_full_size():
    g = C.cl()
    counts, V = gpu_vertex(g, validate=False)
    gd = golden("cl")
    assert gd is not None and counts == [int(x) for x in gd["counts"]]
    check_vertex_sums(g, counts, V)
    # triangles at sampled vertices from the per-edge definition
    vs = _sampled_vertices(g, 200, 23)
    eu, ev = oracle.edges(g)
    for v in vs[:40]:
        sel = (eu == v) | (ev == v)
        if sel.any():
            T, _, _ = oracle.per_edge(g, eu[sel], ev[sel])
            assert int(V[v, 2]) == int(T.sum()) // 2


def test_vertex_counts_rmat22_full_size():
    # the bench configuration: n = 2^22 is within the 64-bit bound
    gd = golden("rmat")
    if gd is None:
        pytest.skip("R-MAT oracle counts not generated yet")
    g = C.rmat22()
    counts, V = gpu_vertex(g, validate=False)
    assert counts == [int(x) for x in gd["counts"]]
    check_vertex_sums(g, counts, V)
    d = g.degrees()
    iso = np.nonzero(d == 0)[0][:5]
    # an isolated vertex v extends each 3-subset of G - v by one independent
    # vertex; G - v has G's triangles and 2-stars, and G's 1-edge 3-subsets
    # minus the m that contain v
    for v in iso:
        r = V[v].astype(object)
        assert r[0] == 0 and r[2] == 0 and r[3] == 0 and r[4] == counts[0]
        assert r[12] == counts[2] and r[13] == counts[3] and r[15] == counts[4] - counts[0]
    eu, ev = oracle.edges(g)
    for v in _sampled_vertices(g, 30, 29)[:12]:
        sel = (eu == v) | (ev == v)
        if sel.any() and d[v] < 2000:
            T, _, _ = oracle.per_edge(g, eu[sel], ev[sel])
            assert int(V[v, 2]) == int(T.sum()) // 2


def test_vertex_counts_reject_too_many_vertices():
    import torch

    n = 4_900_000  # C(n - 1, 3) > 2^64
    rp = torch.zeros(n + 1, dtype=torch.int32, device="cuda:0")
    col = torch.zeros(0, dtype=torch.int32, device="cuda:0")
    with pytest.raises(gl.GraphletError) as e:
        gl.graphlet_count_vertex(rp, col, n)
    assert e.value.code == -5


# ------------------------------------------------------------ edge updates


def _toggle(g, a, b):
    eu, ev = oracle.edges(g)
    edges = set(zip(eu.tolist(), ev.tolist()))
    key = (min(a, b), max(a, b))
    present = key in edges
    (edges.discard if present else edges.add)(key)
    return graphgen.from_edges(g.n, sorted(edges)), not present


@pytest.mark.parametrize("seed", range(3))
def test_edge_update_chains_vs_recount(seed):
    rng = np.random.default_rng(5000 + seed)
    n = int(rng.integers(8, 50))
    g = rand_graph(rng, n, float(rng.uniform(0.05, 0.6)))
    counts = oracle.bruteforce(g)
    for step in range(25):
        a, b = map(int, rng.choice(n, 2, replace=False))
        g2, inserted = _toggle(g, a, b)
        counts = gl.graphlet_update_edge(dev(g.row_ptr), dev(g.col), g.n, a, b, inserted, counts)
        g = g2
        assert counts == oracle.bruteforce(g), step


def test_edge_update_hub_edges():
    g = graphgen.rmat(13, 16, 0.57, 0.19, 0.19, 12)
    counts = gpu_counts(g, validate=False)
    d = g.degrees()
    hubs = np.argsort(-d)[:6].tolist()
    eu, ev = oracle.edges(g)
    pairs = [(hubs[0], int(g.col[g.row_ptr[hubs[0]]]))]  # an edge at the top hub
    pairs += [(hubs[i], hubs[j]) for i in range(3) for j in range(i + 1, 6)][:4]
    for a, b in pairs:
        g2, inserted = _toggle(g, a, b)
        counts = gl.graphlet_update_edge(dev(g.row_ptr), dev(g.col), g.n, a, b, inserted, counts)
        g = g2
        assert counts == gpu_counts(g, validate=False)
    assert counts == oracle.identity_route(g)


def test_edge_update_rejects_bad_requests():
    g = graphgen.from_edges(6, [(0, 1), (1, 2), (2, 3)])
    c = oracle.bruteforce(g)
    rp, col = dev(g.row_ptr), dev(g.col)
    for a, b, ins in [(0, 1, True), (0, 2, False), (3, 3, True), (0, 9, True)]:
        with pytest.raises(gl.GraphletError) as e:
            gl.graphlet_update_edge(rp, col, g.n, a, b, ins, c)
        assert e.value.code == -1


# ------------------------------------------------------------ API behaviour


def test_validation_rejects_bad_csr():
    import torch

    def call(n, rp, col):
        with pytest.raises(gl.GraphletError) as e:
            gl.graphlet_count(dev(np.array(rp, np.int32)), dev(np.array(col, np.int32)), n,
                              validate=True)
        return e.value.code

    assert call(3, [0, 2, 3, 4], [2, 1, 0, 0]) == -2  # unsorted row 0
    assert call(2, [0, 2, 4], [0, 1, 0, 1]) == -3  # self loops, symmetric
    assert call(3, [0, 1, 1, 2], [1, 0]) == -4  # 0->1 but 1 has no list entry
    assert call(2, [0, 1, 2], [5, 0]) == -4  # id out of range
    torch.cuda.synchronize()


def test_unvalidated_asymmetric_csr_is_rejected():
    # without GC_VALIDATE the prepass still refuses a CSR whose entries lack
    # their reverse (reverse search from upper entries plus the count of
    # lower entries), and every kernel stays in bounds on the way
    import torch

    cases = [
        (3, [0, 1, 1, 2], [1, 0]),              # no reverse at all
        (3, [0, 1, 3, 4], [1, 0, 2, 0]),        # 1->2 and 2->0 unpaired
        (4, [0, 2, 3, 4, 6], [1, 2, 0, 3, 0, 1]),  # four unpaired entries
    ]
    for n, rp, col in cases:
        with pytest.raises(gl.GraphletError) as e:
            gl.graphlet_count(dev(np.array(rp, np.int32)), dev(np.array(col, np.int32)), n)
        assert e.value.code == -4, (rp, col)
    torch.cuda.synchronize()
    # a valid graph right after is unaffected
    g = graphgen.from_edges(6, [(0, 1), (1, 2), (2, 0), (3, 4)])
    assert gpu_counts(g, validate=False) == oracle.bruteforce(g)


def test_explicit_workspace():
    import torch

    g = graphgen.er_gnm(1000, 8000, 31)
    rp, col = dev(g.row_ptr), dev(g.col)
    need = gl.graphlet_workspace_size(rp, col, g.n, per_edge=True)
    ws = torch.empty(need, dtype=torch.uint8, device="cuda:0")
    c, pe = gl.graphlet_count(rp, col, g.n, per_edge=True, workspace=ws)
    assert c == oracle.identity_route(g)
    small = torch.empty(need // 2, dtype=torch.uint8, device="cuda:0")
    with pytest.raises(gl.GraphletError) as e:
        gl.graphlet_count(rp, col, g.n, per_edge=True, workspace=small)
    assert e.value.code == -6


@pytest.mark.parametrize("per_edge", [0, 1, 2])
def test_host_only_workspace_bound_suffices(per_edge):
    # the bound from n and nnz alone covers the degree-aware size, and a
    # workspace of exactly the bound runs every mode
    import torch

    for g in (graphgen.er_gnm(1000, 8000, 31), graphgen.rmat(12, 16, 0.57, 0.19, 0.19, 5),
              hub_lists_graph(2500)):
        rp, col = dev(g.row_ptr), dev(g.col)
        bound = gl.graphlet_workspace_bound(g.n, len(g.col), per_edge)
        assert bound >= gl.graphlet_workspace_size(rp, col, g.n, per_edge=per_edge)
        ws = torch.empty(bound, dtype=torch.uint8, device="cuda:0")
        want = oracle.identity_route(g)
        if per_edge == 2:
            c, _ = gl.graphlet_count_local(rp, col, g.n, workspace=ws)
        elif per_edge == 1:
            c, _ = gl.graphlet_count(rp, col, g.n, per_edge=True, workspace=ws)
        else:
            c = gl.graphlet_count(rp, col, g.n, workspace=ws)
        assert c == want


# ------------------------------------------------------------ batched


def batched_gpu(b):
    out = gl.graphlet_count_batched(dev(b.node_off), dev(b.row_ptr), dev(b.col))
    return out.cpu().numpy()


def make_batch(graphs):
    node_off = [0]
    rp = [0]
    cols = []
    for g in graphs:
        base = rp[-1]
        rp.extend((base + g.row_ptr[1:]).tolist())
        cols.append(g.col)
        node_off.append(node_off[-1] + g.n)
    col = np.concatenate(cols) if cols else np.zeros(0, np.int32)
    return graphgen.Batch(np.array(node_off, np.int64), np.zeros(len(graphs), np.int64),
                          np.array(rp, np.int32), col.astype(np.int32))


def test_batched_mixed_sizes_vs_oracle():
    rng = np.random.default_rng(77)
    graphs = []
    for n in [0, 1, 2, 3, 4, 5, 17, 64, 65, 200, 256, 257, 400, 640, 641, 800, 1024]:
        graphs.append(rand_graph(rng, n, float(rng.uniform(0.02, 0.3))))
    graphs.append(graphgen.rgg_torus(500, 8.0, 3))
    graphs.append(graphgen.from_edges(30, [(a, b) for a in range(30) for b in range(a + 1, 30)]))
    b = make_batch(graphs)
    out = batched_gpu(b)
    for i, g in enumerate(graphs):
        assert out[i].tolist() == oracle.identity_route(g), i


def batch8192_oracle_counts(b):
    """The oracle's counts of every graph of the 8192-graph batch, stored by
    tests/golden/make_golden.py (identity route, one graph at a time)."""
    gd = golden("batch8192")
    assert gd is not None, "batch8192 oracle counts not generated"
    assert gd["sha256"] == b.sha256() and gd["graphs"] == b.graphs
    with np.load(os.path.join(HERE, "golden", gd["counts_file"])) as z:
        want = z["counts"]
    h = hashlib.sha256(np.ascontiguousarray(want, dtype="<i8").tobytes()).hexdigest()
    assert h == gd["counts_sha256"]
    return want


def test_batched_config4_every_graph_vs_oracle():
    # all 8192 x 17 entries, for the one-shot call and for the autotuned plan
    # replayed as a HIP graph (the form the benchmark times)
    b = C.batch8192()
    want = batch8192_oracle_counts(b)
    # spot check: the stored matrix is the oracle's
    rng = np.random.default_rng(4)
    for i in rng.choice(b.graphs, 8, replace=False):
        assert want[i].tolist() == oracle.identity_route(b.graph(int(i))), i
    nd, rp, col = dev(b.node_off), dev(b.row_ptr), dev(b.col)
    out = gl.graphlet_count_batched(nd, rp, col).cpu().numpy()
    bad = np.nonzero((out != want).any(1))[0]
    assert len(bad) == 0, f"{len(bad)} graphs differ, first {bad[:10].tolist()}"
    with gl.BatchPlan(nd, rp, col, tune=True) as plan:
        for rep in range(2):
            plan.out.zero_()
            got = plan.run().cpu().numpy()
            bad = np.nonzero((got != want).any(1))[0]
            assert len(bad) == 0, f"replay {rep}: {len(bad)} graphs differ, first {bad[:10]}"


def test_batched_equals_single_graph_path():
    b = C.batch8192(64)
    out = batched_gpu(b)
    for i in range(b.graphs):
        g = b.graph(i)
        assert out[i].tolist() == gpu_counts(g, validate=False)


def test_batched_rejects_oversized_graph():
    g = graphgen.from_edges(1100, [(0, 1)])
    b = make_batch([g])
    with pytest.raises(gl.GraphletError) as e:
        batched_gpu(b)
    assert e.value.code == -5


def test_batch_gfd_exact():
    b = C.batch8192(300)
    counts = gl.graphlet_count_batched(dev(b.node_off), dev(b.row_ptr), dev(b.col))
    c = counts.cpu().numpy()
    n = np.diff(b.node_off)
    for connected in (False, True):
        got = gl.graphlet_batch_gfd(counts, connected_only=connected).cpu().numpy()
        want = np.zeros(c.shape)
        for lo, hi, hc in ((0, 2, 1), (2, 6, 4), (6, 17, 12)):
            top = hc if connected else hi
            s = c[:, lo:top].sum(1).astype(np.float64)
            with np.errstate(invalid="ignore", divide="ignore"):
                q = c[:, lo:top].astype(np.float64) / s[:, None]
            want[:, lo:top] = np.where(s[:, None] > 0, q, 0.0)
        np.testing.assert_array_equal(got, want)
        if not connected:  # all classes: the size-k sums are C(n, k)
            np.testing.assert_array_equal(c[:, 6:17].sum(1), n * (n - 1) * (n - 2) * (n - 3) // 24)


# ------------------------------------------------------------ batched per-vertex counts


def batch_vertex_gpu(b, validate=True):
    out = gl.graphlet_batch_vertex(dev(b.node_off), dev(b.row_ptr), dev(b.col),
                                   validate=validate)
    return out.cpu().numpy()


def check_batch_vertex_sums(b, counts, V):
    # per graph: summed over its vertices, a size-k class is seen k times;
    # each vertex's row is a census of the subsets containing it
    for i in range(b.graphs):
        a, e = int(b.node_off[i]), int(b.node_off[i + 1])
        n = e - a
        Vi = V[a:e].astype(np.int64)
        np.testing.assert_array_equal(Vi.sum(0), np.array(oracle.CLASS_K) * counts[i])
        if n:
            np.testing.assert_array_equal(Vi[:, 0], np.diff(b.row_ptr[a:e + 1]))
            assert (Vi[:, :2].sum(1) == n - 1).all()
            assert (Vi[:, 2:6].sum(1) == comb(n - 1, 2)).all()
            assert (Vi[:, 6:].sum(1) == comb(n - 1, 3)).all()


def test_batch_vertex_mixed_sizes_vs_oracle():
    rng = np.random.default_rng(91)
    graphs = []
    for n in [0, 1, 2, 3, 4, 5, 9, 17, 33, 60, 64, 65, 128, 129, 256, 257, 512, 513, 1024]:
        graphs.append(rand_graph(rng, n, float(rng.uniform(0.02, 0.35))))
    graphs.append(graphgen.from_edges(50, [(a, b) for a in range(50) for b in range(a + 1, 50)]))
    graphs.append(graphgen.from_edges(300, [(0, i) for i in range(1, 300)]))
    graphs.append(graphgen.rgg_torus(400, 8.0, 9))
    b = make_batch(graphs)
    V = batch_vertex_gpu(b)
    assert V.shape == (int(b.node_off[-1]), 17)
    counts = batched_gpu(b)
    check_batch_vertex_sums(b, counts, V)
    for i, g in enumerate(graphs):
        Vi = V[b.node_off[i]:b.node_off[i + 1]]
        if g.n <= 60:
            np.testing.assert_array_equal(Vi, oracle.vertex_bruteforce(g).astype(np.uint64))
        else:
            vs = _sampled_vertices(g, 12, 100 + i)
            np.testing.assert_array_equal(Vi[vs], oracle.vertex_by_deletion(g, vs))


def test_batch_vertex_config4_sample():
    b = C.batch8192()
    V = batch_vertex_gpu(b, validate=False)
    counts = batched_gpu(b)
    check_batch_vertex_sums(b, counts, V)
    rng = np.random.default_rng(41)
    for i in rng.choice(b.graphs, 24, replace=False):
        g = b.graph(int(i))
        Vi = V[b.node_off[i]:b.node_off[i + 1]]
        vs = _sampled_vertices(g, 6, int(i))
        np.testing.assert_array_equal(Vi[vs], oracle.vertex_by_deletion(g, vs))


def test_batch_vertex_equals_single_graph_path():
    b = C.batch8192(48)
    V = batch_vertex_gpu(b)
    for i in range(b.graphs):
        _, Vg = gpu_vertex(b.graph(i), validate=False)
        np.testing.assert_array_equal(V[b.node_off[i]:b.node_off[i + 1]], Vg)


def test_batch_vertex_degenerate_batches():
    import torch

    # no graphs: nothing to do
    empty = make_batch([])
    assert batch_vertex_gpu(empty).shape == (0, 17)
    # only vertex-free graphs: nothing written
    b = make_batch([graphgen.from_edges(0, []), graphgen.from_edges(0, [])])
    assert batch_vertex_gpu(b).shape == (0, 17)
    # edgeless graphs: every vertex sits in the fully disconnected classes only
    b = make_batch([graphgen.from_edges(7, []), graphgen.from_edges(0, []),
                    graphgen.from_edges(2, [(0, 1)])])
    V = batch_vertex_gpu(b)
    want = np.zeros((9, 17), np.uint64)
    want[:7, 1], want[:7, 5], want[:7, 16] = 6, 15, 20
    want[7:, 0] = 1
    np.testing.assert_array_equal(V, want)
    # a caller's buffer that is too small is refused before the call
    with pytest.raises(ValueError):
        gl.graphlet_batch_vertex(dev(b.node_off), dev(b.row_ptr), dev(b.col),
                                 out=torch.empty((2, 17), dtype=torch.uint64, device="cuda:0"))


def test_batch_vertex_concurrent_callers():
    # two host threads, each on a stream of its own, share the library's
    # class streams: every call must still equal the single-threaded result
    import threading

    import torch

    b1, b2 = C.batch8192(96), make_batch([rand_graph(np.random.default_rng(s), n, 0.2)
                                          for s, n in enumerate([30, 70, 150, 300, 600, 900])])
    want = [batch_vertex_gpu(b1), batch_vertex_gpu(b2)]
    dev_b = [tuple(dev(x) for x in (b.node_off, b.row_ptr, b.col)) for b in (b1, b2)]
    got, errs = [[], []], []

    def worker(k):
        try:
            st = torch.cuda.Stream()
            for _ in range(4):
                out = gl.graphlet_batch_vertex(*dev_b[k], stream=st)
                got[k].append(out.cpu().numpy())
        except Exception as e:  # reported below, on the main thread
            errs.append(e)

    ts = [threading.Thread(target=worker, args=(k,)) for k in (0, 1)]
    for t in ts:
        t.start()
    for t in ts:
        t.join()
    assert not errs, errs
    for k in (0, 1):
        assert len(got[k]) == 4
        for g in got[k]:
            np.testing.assert_array_equal(g, want[k])


def test_batch_vertex_rejects_invalid_batches():
    g = graphgen.from_edges(1100, [(0, 1)])
    with pytest.raises(gl.GraphletError) as e:
        batch_vertex_gpu(make_batch([g]))
    assert e.value.code == -5
    # an asymmetric list (0 -> 1 without 1 -> 0, padded to an even length)
    bad = graphgen.Batch(np.array([0, 3], np.int64), np.zeros(1, np.int64),
                         np.array([0, 2, 2, 2], np.int32), np.array([1, 2], np.int32))
    with pytest.raises(gl.GraphletError):
        batch_vertex_gpu(bad, validate=True)


# ------------------------------------------------------------ batched plans

CLASS_SETS = [[16], [4, 16], [1, 4, 16], [4, 10, 16], [2, 6, 10, 16], [1, 2, 4, 6, 8, 10, 12, 16]]
SHAPES = [(blk, cls) for blk in (256, 512) for cls in CLASS_SETS]


def mixed_batch_graphs(seed=78):
    rng = np.random.default_rng(seed)
    graphs = []
    for n in [0, 1, 2, 3, 5, 17, 40, 63, 64, 65, 100, 127, 128, 129, 191, 192, 193, 255, 256,
              257, 300, 400, 640, 641, 1024]:
        graphs.append(rand_graph(rng, n, float(rng.uniform(0.02, 0.4))))
    graphs.append(graphgen.rgg_torus(150, 8.0, 5))
    graphs.append(graphgen.from_edges(70, [(a, b) for a in range(70) for b in range(a + 1, 70)]))
    return graphs


def test_batch_plan_every_shape_vs_oracle():
    graphs = mixed_batch_graphs()
    want = [oracle.identity_route(g) for g in graphs]
    b = make_batch(graphs)
    with gl.BatchPlan(dev(b.node_off), dev(b.row_ptr), dev(b.col), tune=False) as plan:
        for blk, cls in SHAPES:
            plan.reshape(blk, cls)
            info = plan.info()
            assert info["block"] == blk and set(info["class_words"]) <= set(cls)
            assert sum(info["class_graphs"]) == len(graphs)
            out = plan.run().cpu().numpy()
            for i, g in enumerate(graphs):
                assert out[i].tolist() == want[i], (blk, cls, i)
        with pytest.raises(gl.GraphletError) as e:
            plan.reshape(256, [4, 10])  # nothing holds the n = 1024 graph
        assert e.value.code == -1


def test_batch_plan_tuned_replays_match_eager():
    import torch

    b = C.batch8192(512)
    nd, rp, col = dev(b.node_off), dev(b.row_ptr), dev(b.col)
    eager = gl.graphlet_count_batched(nd, rp, col).cpu().numpy()
    with gl.BatchPlan(nd, rp, col, tune=True) as plan:
        info = plan.info()
        assert info["candidates"] > 0 and info["tuned_ms"] > 0
        for rep in range(4):
            plan.out.zero_()                      # eager work between the replays
            x = torch.randn(1 << 20, device="cuda:0")
            (x * x).sum().item()
            torch.cuda.synchronize()
            got = plan.run().cpu().numpy()
            np.testing.assert_array_equal(got, eager, err_msg=f"replay {rep}")
    rng = np.random.default_rng(5)
    for i in rng.choice(b.graphs, 40, replace=False):
        assert eager[i].tolist() == oracle.identity_route(b.graph(int(i))), i


def test_batch_plan_new_contents_same_sizes():
    rng = np.random.default_rng(79)
    sizes = [30, 90, 250, 500]
    g1 = [rand_graph(rng, n, 0.2) for n in sizes]
    b1 = make_batch(g1)
    nd, rp, col = dev(b1.node_off), dev(b1.row_ptr), dev(b1.col)
    with gl.BatchPlan(nd, rp, col, tune=False) as plan:
        assert plan.run().cpu().numpy().tolist() == [oracle.identity_route(g) for g in g1]
        # relabel every graph: same n and nnz per graph, new adjacency lists
        g2 = []
        for g in g1:
            perm = rng.permutation(g.n)
            eu, ev = oracle.edges(g)
            g2.append(graphgen.from_edges(g.n, list(zip(perm[eu], perm[ev]))))
        b2 = make_batch(g2)
        assert (b2.node_off == b1.node_off).all() and b2.col.shape == b1.col.shape
        rp.copy_(dev(b2.row_ptr))
        col.copy_(dev(b2.col))
        assert plan.run().cpu().numpy().tolist() == [oracle.identity_route(g) for g in g2]


def test_batch_plan_rejects_graph_grown_beyond_its_class():
    rng = np.random.default_rng(80)
    small, big = rand_graph(rng, 50, 0.2), rand_graph(rng, 300, 0.1)
    b1 = make_batch([small, big])
    b2 = make_batch([big, small])  # same total rows and entries, bins swapped
    assert b1.row_ptr.shape == b2.row_ptr.shape and b1.col.shape == b2.col.shape
    nd, rp, col = dev(b1.node_off), dev(b1.row_ptr), dev(b1.col)
    with gl.BatchPlan(nd, rp, col, tune=False) as plan:
        plan.reshape(256, [1, 16])
        plan.run()
        nd.copy_(dev(b2.node_off))
        rp.copy_(dev(b2.row_ptr))
        col.copy_(dev(b2.col))
        with pytest.raises(gl.GraphletError) as e:
            plan.run()
        assert e.value.code == -1
        plan.reshape(256, [1, 16])  # a new layout for the new contents
        out = plan.run().cpu().numpy()
    assert out[0].tolist() == oracle.identity_route(big)
    assert out[1].tolist() == oracle.identity_route(small)
