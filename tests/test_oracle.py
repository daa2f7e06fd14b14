"""Pins for the CPU oracle against things other than itself.

Each route of the oracle is checked against what the paper and plain
combinatorics fix: Table 1's printed properties for every graphlet, closed
forms for named graph families, the complement relation of Section 2, the
effect of adding an isolated vertex, relabelling invariance, and agreement
between routes that share no code (subset brute force, non-induced inversion,
per-edge definition).
"""
import itertools
import os
from math import comb

import numpy as np
import pytest

import graphgen
import oracle

HERE = os.path.dirname(os.path.abspath(__file__))
IDX = {name: i for i, name in enumerate(oracle.NAMES)}


def load_table1():
    rows = {}
    with open(os.path.join(HERE, "golden", "table1.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            gid, name, rho, delta, dbar, tri, diam, comp, compl = line.split()
            rows[gid] = dict(name=name, rho=float(rho), delta=int(delta), dbar=float(dbar),
                             tri=int(tri), diam=None if diam == "inf" else int(diam),
                             comp=int(comp), compl=compl)
    return rows


TABLE1 = load_table1()

# Each graphlet drawn from its Table 1 name, on vertices 0..k-1.
SHAPES = {
    "g4_1": (4, [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)]),  # 4-clique
    "g4_2": (4, [(0, 1), (1, 2), (2, 3), (3, 0), (0, 2)]),  # 4-cycle plus one chord
    "g4_3": (4, [(0, 1), (1, 2), (2, 0), (2, 3)]),  # triangle with a tail
    "g4_4": (4, [(0, 1), (1, 2), (2, 3), (3, 0)]),  # 4-cycle
    "g4_5": (4, [(0, 1), (0, 2), (0, 3)]),  # 3-star
    "g4_6": (4, [(0, 1), (1, 2), (2, 3)]),  # 4-path
    "g4_7": (4, [(0, 1), (1, 2), (2, 0)]),  # triangle + isolated node
    "g4_8": (4, [(0, 1), (0, 2)]),  # 2-star + isolated node
    "g4_9": (4, [(0, 1), (2, 3)]),  # two disjoint edges
    "g4_10": (4, [(0, 1)]),  # one edge + two isolated nodes
    "g4_11": (4, []),  # independent set
    "g3_1": (3, [(0, 1), (1, 2), (2, 0)]),
    "g3_2": (3, [(0, 1), (0, 2)]),
    "g3_3": (3, [(0, 1)]),
    "g3_4": (3, []),
    "g2_1": (2, [(0, 1)]),
    "g2_2": (2, []),
}


def props(n, edges):
    """rho, Delta, dbar, triangles, diameter of the largest component, components."""
    adj = {v: set() for v in range(n)}
    for a, b in edges:
        adj[a].add(b)
        adj[b].add(a)
    deg = [len(adj[v]) for v in range(n)]
    tri = sum(1 for a, b, c in itertools.combinations(range(n), 3)
              if b in adj[a] and c in adj[a] and c in adj[b])
    seen, comps = set(), []
    for s in range(n):
        if s in seen:
            continue
        comp, stack = {s}, [s]
        while stack:
            x = stack.pop()
            for y in adj[x]:
                if y not in comp:
                    comp.add(y)
                    stack.append(y)
        seen |= comp
        comps.append(comp)
    big = max(comps, key=len)
    if len(big) == 1:
        diam = None
    else:
        diam = 0
        for s in big:
            dist, frontier = {s: 0}, [s]
            while frontier:
                nxt = []
                for x in frontier:
                    for y in adj[x]:
                        if y not in dist:
                            dist[y] = dist[x] + 1
                            nxt.append(y)
                frontier = nxt
            diam = max(diam, max(dist.values()))
    return (round(len(edges) / comb(n, 2), 2), max(deg), round(2 * len(edges) / n, 2), tri,
            diam, len(comps))


def counts_of(n, edges, route=oracle.bruteforce):
    return route(graphgen.from_edges(n, edges))


def complement(n, edges):
    es = {(min(a, b), max(a, b)) for a, b in edges}
    return [(a, b) for a in range(n) for b in range(a + 1, n) if (a, b) not in es]


def rand_graph(rng, n, p):
    return [(a, b) for a in range(n) for b in range(a + 1, n) if rng.random() < p]


# --------------------------------------------------------------------- Table 1


@pytest.mark.parametrize("gid", sorted(SHAPES))
def test_shape_matches_table1_row(gid):
    n, edges = SHAPES[gid]
    row = TABLE1[gid]
    rho, delta, dbar, tri, diam, comp = props(n, edges)
    assert rho == pytest.approx(row["rho"], abs=0.006)
    assert delta == row["delta"]
    assert dbar == pytest.approx(row["dbar"], abs=0.006)
    assert tri == row["tri"]
    assert diam == row["diam"]
    assert comp == row["comp"]


@pytest.mark.parametrize("gid", sorted(SHAPES))
def test_each_graphlet_counts_itself_once(gid):
    n, edges = SHAPES[gid]
    c = counts_of(n, edges)
    k = int(gid[1])
    block = {2: range(0, 2), 3: range(2, 6), 4: range(6, 17)}[k]
    for i in block:
        assert c[i] == (1 if i == IDX[gid] else 0), (gid, oracle.NAMES[i], c)


def test_classifier_rows_are_distinct_and_complete():
    # Every 4-vertex graph (64 edge subsets) lands on exactly one Table 1 row,
    # and each of the 11 rows is hit.
    hit = set()
    pairs = list(itertools.combinations(range(4), 2))
    for mask in range(64):
        edges = [pairs[i] for i in range(6) if mask >> i & 1]
        c = counts_of(4, edges)
        assert sum(c[6:]) == 1
        hit.add(int(np.argmax(c[6:])))
    assert hit == set(range(11))


def test_classify4_table_unknown_row():
    assert oracle.classify4(4, 4, 1) == -1
    assert oracle.classify4(6, 3, 1) == 0
    assert oracle.classify4(0, 0, 4) == 10


# ----------------------------------------------------------------- closed forms


@pytest.mark.parametrize("n", [0, 1, 2, 3, 4, 5, 9])
def test_complete_graph(n):
    c = counts_of(n, list(itertools.combinations(range(n), 2)))
    want = [0] * 17
    want[IDX["g2_1"]] = comb(n, 2)
    want[IDX["g3_1"]] = comb(n, 3)
    want[IDX["g4_1"]] = comb(n, 4)
    assert c == want


@pytest.mark.parametrize("n", [0, 1, 3, 7, 12])
def test_empty_graph(n):
    c = counts_of(n, [])
    want = [0] * 17
    want[IDX["g2_2"]] = comb(n, 2)
    want[IDX["g3_4"]] = comb(n, 3)
    want[IDX["g4_11"]] = comb(n, 4)
    assert c == want


@pytest.mark.parametrize("leaves", [1, 2, 3, 4, 8])
def test_star(leaves):
    # centre 0 joined to every leaf: every 3-set with the centre is a 2-star,
    # every 4-set with the centre a 3-star, sets of leaves only are empty.
    n = leaves + 1
    c = counts_of(n, [(0, i) for i in range(1, n)])
    want = [0] * 17
    want[IDX["g2_1"]] = leaves
    want[IDX["g2_2"]] = comb(leaves, 2)
    want[IDX["g3_2"]] = comb(leaves, 2)
    want[IDX["g3_4"]] = comb(leaves, 3)
    want[IDX["g4_5"]] = comb(leaves, 3)
    want[IDX["g4_11"]] = comb(leaves, 4)
    assert c == want


@pytest.mark.parametrize("n", [6, 7, 10])
def test_cycle(n):
    # C_n: consecutive triples are 2-stars, consecutive quadruples 4-paths;
    # an edge plus a vertex away from both ends: n (n - 4); a 2-path plus a
    # vertex away from all three: n (n - 5); two edges with no edge between:
    # n (n - 5) / 2.
    c = counts_of(n, [(i, (i + 1) % n) for i in range(n)])
    assert c[IDX["g2_1"]] == n
    assert c[IDX["g3_1"]] == 0
    assert c[IDX["g3_2"]] == n
    assert c[IDX["g3_3"]] == n * (n - 4)
    assert c[IDX["g4_6"]] == n
    assert c[IDX["g4_4"]] == 0 and c[IDX["g4_5"]] == 0
    assert c[IDX["g4_8"]] == n * (n - 5)
    assert c[IDX["g4_9"]] == n * (n - 5) // 2


def test_small_cycles():
    assert counts_of(4, [(0, 1), (1, 2), (2, 3), (3, 0)])[IDX["g4_4"]] == 1
    assert counts_of(5, [(i, (i + 1) % 5) for i in range(5)])[IDX["g4_6"]] == 5


@pytest.mark.parametrize("n", [5, 6, 11])
def test_path(n):
    c = counts_of(n, [(i, i + 1) for i in range(n - 1)])
    assert c[IDX["g3_2"]] == n - 2
    assert c[IDX["g4_6"]] == n - 3
    assert c[IDX["g4_5"]] == 0 and c[IDX["g4_4"]] == 0


@pytest.mark.parametrize("a,b", [(2, 2), (2, 3), (3, 4), (1, 5)])
def test_complete_bipartite(a, b):
    # K_{a,b}: 4-cycles are 2+2 vertex choices; 3-stars are 1+3 choices.
    edges = [(i, a + j) for i in range(a) for j in range(b)]
    c = counts_of(a + b, edges)
    assert c[IDX["g3_1"]] == 0
    assert c[IDX["g4_4"]] == comb(a, 2) * comb(b, 2)
    assert c[IDX["g4_5"]] == a * comb(b, 3) + b * comb(a, 3)
    assert c[IDX["g4_1"]] == c[IDX["g4_2"]] == c[IDX["g4_3"]] == 0


@pytest.mark.parametrize("k", [2, 3, 5])
def test_perfect_matching(k):
    n = 2 * k
    c = counts_of(n, [(2 * i, 2 * i + 1) for i in range(k)])
    assert c[IDX["g4_9"]] == comb(k, 2)
    assert c[IDX["g3_3"]] == k * (n - 2)
    assert c[IDX["g4_10"]] == k * (comb(n - 2, 2) - (k - 1))


# ------------------------------------------------------------------ invariants

PI = {gid: row["compl"] for gid, row in TABLE1.items()}


@pytest.mark.parametrize("seed", range(12))
def test_complement_relation(seed):
    # Section 2: f(g, G) = f(complement of g, complement of G).
    rng = np.random.default_rng(seed)
    n = int(rng.integers(4, 11))
    edges = rand_graph(rng, n, rng.random())
    c = counts_of(n, edges)
    cc = counts_of(n, complement(n, edges))
    for gid in oracle.NAMES:
        assert cc[IDX[gid]] == c[IDX[PI[gid]]], gid


@pytest.mark.parametrize("seed", range(10))
def test_sums_and_isolated_vertex(seed):
    rng = np.random.default_rng(100 + seed)
    n = int(rng.integers(1, 11))
    edges = rand_graph(rng, n, rng.random())
    c = counts_of(n, edges)
    assert c[0] + c[1] == comb(n, 2)
    assert sum(c[2:6]) == comb(n, 3)
    assert sum(c[6:]) == comb(n, 4)
    d = counts_of(n + 1, edges)
    delta = [d[i] - c[i] for i in range(17)]
    want = [0] * 17
    want[IDX["g2_2"]] = n
    want[IDX["g3_3"]] = c[IDX["g2_1"]]
    want[IDX["g3_4"]] = c[IDX["g2_2"]]
    want[IDX["g4_7"]] = c[IDX["g3_1"]]
    want[IDX["g4_8"]] = c[IDX["g3_2"]]
    want[IDX["g4_10"]] = c[IDX["g3_3"]]
    want[IDX["g4_11"]] = c[IDX["g3_4"]]
    assert delta == want


@pytest.mark.parametrize("seed", range(6))
def test_relabelling_invariance(seed):
    rng = np.random.default_rng(200 + seed)
    n = int(rng.integers(5, 12))
    edges = rand_graph(rng, n, 0.45)
    perm = rng.permutation(n)
    moved = [(int(perm[a]), int(perm[b])) for a, b in edges]
    assert counts_of(n, edges) == counts_of(n, moved)
    assert counts_of(n, edges, oracle.identity_route) == counts_of(n, moved, oracle.identity_route)


# ------------------------------------------------------- routes against routes


def _families(rng):
    yield "er", int(rng.integers(0, 14)), None
    n = int(rng.integers(4, 13))
    yield "dense", n, rand_graph(rng, n, 0.8)
    n = int(rng.integers(4, 13))
    yield "sparse", n, rand_graph(rng, n, 0.15)


@pytest.mark.parametrize("seed", range(40))
def test_identity_route_equals_bruteforce(seed):
    rng = np.random.default_rng(300 + seed)
    for kind, n, edges in _families(rng):
        if edges is None:
            edges = rand_graph(rng, n, rng.random())
        g = graphgen.from_edges(n, edges)
        assert oracle.identity_route(g) == oracle.bruteforce(g), (kind, n, edges)


def test_identity_route_equals_bruteforce_structured():
    # stars of cliques, bipartite, geometric and a small power law
    cases = []
    k5 = list(itertools.combinations(range(5), 2))
    soc = k5 + [(a + 5, b + 5) for a, b in k5] + [(0, 10), (5, 10), (10, 11), (10, 12)]
    cases.append((13, soc))
    cases.append((9, [(i, 4 + j) for i in range(4) for j in range(5)]))
    g = graphgen.rgg_torus(60, 8.0, 7)
    cases.append((g.n, list(zip(*oracle.edges(g)))))
    g = graphgen.chung_lu(80, 2.1, 1.0, 300, 5)
    cases.append((g.n, list(zip(*oracle.edges(g)))))
    for n, edges in cases:
        g = graphgen.from_edges(n, edges)
        assert oracle.identity_route(g) == oracle.bruteforce(g)


@pytest.mark.parametrize("seed", range(25))
def test_per_edge_equals_subset_enumeration(seed):
    rng = np.random.default_rng(400 + seed)
    n = int(rng.integers(2, 13))
    g = graphgen.from_edges(n, rand_graph(rng, n, rng.random()))
    eu, ev = oracle.edges(g)
    if len(eu) == 0:
        return
    T, K4, C4 = oracle.per_edge(g, eu, ev)
    bk, bc = oracle.bruteforce_edge4(g, eu, ev)
    np.testing.assert_array_equal(K4, bk)
    np.testing.assert_array_equal(C4, bc)
    A = oracle.bruteforce(g)
    # each triangle has 3 edges, each 4-clique 6, each 4-cycle 4
    assert int(T.sum()) == 3 * A[IDX["g3_1"]]
    assert int(K4.sum()) == 6 * A[IDX["g4_1"]]
    assert int(C4.sum()) == 4 * A[IDX["g4_4"]]
    # |Tri_e| by a plain set intersection
    adj = [set(g.col[g.row_ptr[v]:g.row_ptr[v + 1]].tolist()) for v in range(n)]
    for u, v, t in zip(eu, ev, T):
        assert t == len(adj[u] & adj[v])


def test_per_edge_on_medium_graph_sums():
    g = graphgen.er_gnm(300, 6000, 11)
    eu, ev = oracle.edges(g)
    T, K4, C4 = oracle.per_edge(g, eu, ev)
    B = oracle.identity_route(g)
    assert int(T.sum()) == 3 * B[IDX["g3_1"]]
    assert int(K4.sum()) == 6 * B[IDX["g4_1"]]
    assert int(C4.sum()) == 4 * B[IDX["g4_4"]]


def test_oracle_rejects_bad_csr():
    bad = graphgen.Csr(3, np.array([0, 1, 2, 2], np.int32), np.array([1, 2], np.int32))  # asymmetric
    assert oracle.check_csr(bad) != 0
    with pytest.raises(ValueError):
        oracle.identity_route(bad)
    loop = graphgen.Csr(2, np.array([0, 1, 1], np.int32), np.array([0], np.int32))
    assert oracle.check_csr(loop) != 0


def test_wide_counts_exceed_int64():
    # 3-node-independent sets on 2^22 isolated vertices: C(n,3) > 2^63.
    n = 1 << 22
    g = graphgen.Csr(n, np.zeros(n + 1, np.int32), np.zeros(0, np.int32))
    c = oracle.identity_route(g)
    assert c[IDX["g3_4"]] == comb(n, 3) and c[IDX["g3_4"]] > 2**63
    assert c[IDX["g4_11"]] == comb(n, 4)


# ------------------------------------------------------------ per-edge local vectors


def _local_graphs():
    rng = np.random.default_rng(2024)
    out = []
    for _ in range(12):
        n = int(rng.integers(4, 30))
        p = float(rng.random())
        iu = np.triu_indices(n, 1)
        mask = rng.random(len(iu[0])) < p
        out.append(graphgen.from_edges(n, list(zip(iu[0][mask], iu[1][mask]))))
    out.append(graphgen.from_edges(7, [(a, b) for a in range(7) for b in range(a + 1, 7)]))
    out.append(graphgen.from_edges(9, [(0, i) for i in range(1, 9)]))
    out.append(graphgen.from_edges(8, [(i, (i + 1) % 8) for i in range(8)]))
    out.append(graphgen.from_edges(9, [(a, b) for a in range(4) for b in range(4, 9)]))
    return out


@pytest.mark.parametrize("gi", range(16))
def test_edge_local_two_routes_agree(gi):
    g = _local_graphs()[gi]
    eu, ev = oracle.edges(g)
    if len(eu):
        np.testing.assert_array_equal(oracle.edge_local(g, eu, ev),
                                      oracle.edge_local_brute(g, eu, ev))


@pytest.mark.parametrize("gi", range(16))
def test_edge_local_sums(gi):
    # every 3- and 4-subset containing e is counted once; summed over the
    # edges, each graphlet is seen once from each of its edges
    g = _local_graphs()[gi]
    eu, ev = oracle.edges(g)
    if not len(eu):
        return
    L = oracle.edge_local(g, eu, ev)
    n = g.n
    assert (L[:, :3].sum(1) == n - 2).all()
    assert (L[:, 3:].sum(1) == comb(n - 2, 2)).all()
    counts = oracle.bruteforce(g)
    tot = {}
    for j, G in enumerate(oracle.LOCAL_GRAPHLET):
        tot[G] = tot.get(G, 0) + int(L[:, j].sum())
    for G, s in tot.items():
        assert s == oracle.GRAPHLET_EDGES[G] * counts[G], (G, s, counts[G])


def test_edge_local_closed_forms():
    names = oracle.LOCAL_NAMES
    # K_n: every other pair of vertices closes a 4-clique
    n = 8
    g = graphgen.from_edges(n, [(a, b) for a in range(n) for b in range(a + 1, n)])
    L = oracle.edge_local(g, [0], [5])[0]
    want = dict.fromkeys(names, 0)
    want.update(T=n - 2, TT1=comb(n - 2, 2))
    assert dict(zip(names, L.tolist())) == want
    # star with k leaves, edge (centre, leaf): k - 1 star vertices, all pairs 3-stars
    k = 7
    g = graphgen.from_edges(k + 1, [(0, i) for i in range(1, k + 1)])
    L = oracle.edge_local(g, [0], [3])[0]
    want = dict.fromkeys(names, 0)
    want.update(S=k - 1, SS0=comb(k - 1, 2))
    assert dict(zip(names, L.tolist())) == want
    # cycle C_n, edge (0, 1): one star vertex each side, n - 4 others on a path
    n = 11
    g = graphgen.from_edges(n, [(i, (i + 1) % n) for i in range(n)])
    L = oracle.edge_local(g, [0], [1])[0]
    want = dict.fromkeys(names, 0)
    want.update(S=2, I=n - 4, SuSv0=1, SI1=2, SI0=2 * (n - 4) - 2, II1=n - 5,
                II0=comb(n - 4, 2) - (n - 5))
    assert dict(zip(names, L.tolist())) == want


def test_edge_local_planted_mistake_is_caught():
    # a dropped term (the tail edge case) breaks the per-graphlet sum rule
    g = _local_graphs()[3]
    eu, ev = oracle.edges(g)
    L = oracle.edge_local(g, eu, ev)
    L[:, 8] = 0
    counts = oracle.bruteforce(g)
    s = int(L[:, 6].sum() + L[:, 7].sum() + L[:, 8].sum())
    assert counts[8] == 0 or s != 4 * counts[8]


# ------------------------------------------------------------ per-vertex counts


def _vertex_graphs():
    rng = np.random.default_rng(808)
    out = [graphgen.from_edges(1, []), graphgen.from_edges(5, []),
           graphgen.from_edges(2, [(0, 1)]), graphgen.from_edges(3, [(0, 1)])]
    for _ in range(10):
        n = int(rng.integers(4, 22))
        p = float(rng.random())
        iu = np.triu_indices(n, 1)
        mask = rng.random(len(iu[0])) < p
        out.append(graphgen.from_edges(n, list(zip(iu[0][mask], iu[1][mask]))))
    out.append(graphgen.from_edges(7, [(a, b) for a in range(7) for b in range(a + 1, 7)]))
    out.append(graphgen.from_edges(9, [(0, i) for i in range(1, 9)]))
    out.append(graphgen.from_edges(9, [(i, (i + 1) % 9) for i in range(9)]))
    out.append(graphgen.from_edges(10, [(2 * i, 2 * i + 1) for i in range(5)]))
    out.append(graphgen.from_edges(9, [(a, b) for a in range(4) for b in range(4, 9)]))
    return out


N_VERTEX_GRAPHS = 19


@pytest.mark.parametrize("gi", range(N_VERTEX_GRAPHS))
def test_vertex_two_routes_agree(gi):
    # subset enumeration credited to members == g(G) - g(G - v) from the
    # identity route; the two share nothing
    g = _vertex_graphs()[gi]
    np.testing.assert_array_equal(oracle.vertex_bruteforce(g).astype(np.uint64),
                                  oracle.vertex_by_deletion(g))


@pytest.mark.parametrize("gi", range(N_VERTEX_GRAPHS))
def test_vertex_sums(gi):
    # each k-subset is seen once from each of its k members, and the k-subsets
    # holding v are all classified
    g = _vertex_graphs()[gi]
    n = g.n
    V = oracle.vertex_bruteforce(g)
    counts = oracle.bruteforce(g)
    for c in range(17):
        assert int(V[:, c].sum()) == oracle.CLASS_K[c] * counts[c], oracle.NAMES[c]
    assert (V[:, :2].sum(1) == n - 1).all()
    assert (V[:, 2:6].sum(1) == comb(n - 1, 2)).all()
    assert (V[:, 6:].sum(1) == comb(n - 1, 3)).all()


def test_vertex_closed_forms():
    def row(**kw):
        r = [0] * 17
        for k, v in kw.items():
            r[IDX[k]] = v
        return r

    # K_n: every subset is a clique
    n = 7
    V = oracle.vertex_bruteforce(
        graphgen.from_edges(n, [(a, b) for a in range(n) for b in range(a + 1, n)]))
    assert all(list(r) == row(g2_1=n - 1, g3_1=comb(n - 1, 2), g4_1=comb(n - 1, 3)) for r in V)
    # star with L leaves: the centre sees stars only, a leaf also independent sets
    L = 8
    V = oracle.vertex_bruteforce(graphgen.from_edges(L + 1, [(0, i) for i in range(1, L + 1)]))
    assert list(V[0]) == row(g2_1=L, g3_2=comb(L, 2), g4_5=comb(L, 3))
    leaf = row(g2_1=1, g2_2=L - 1, g3_2=L - 1, g3_4=comb(L - 1, 2), g4_5=comb(L - 1, 2),
               g4_11=comb(L - 1, 3))
    assert all(list(r) == leaf for r in V[1:])
    # perfect matching of p edges
    p = 5
    V = oracle.vertex_bruteforce(graphgen.from_edges(2 * p, [(2 * i, 2 * i + 1) for i in range(p)]))
    g49 = p - 1
    g410 = comb(2 * p - 2, 2) - (p - 1) + (p - 1) * (2 * p - 4)
    want = row(g2_1=1, g2_2=2 * p - 2, g3_3=3 * p - 3, g3_4=comb(2 * p - 1, 2) - (3 * p - 3),
               g4_9=g49, g4_10=g410, g4_11=comb(2 * p - 1, 3) - g49 - g410)
    assert all(list(r) == want for r in V)
    # cycle C_9: each vertex is in 3 two-stars and 4 four-paths
    V = oracle.vertex_bruteforce(graphgen.from_edges(9, [(i, (i + 1) % 9) for i in range(9)]))
    assert (V[:, IDX["g3_2"]] == 3).all() and (V[:, IDX["g4_6"]] == 4).all()
    assert (V[:, IDX["g3_1"]] == 0).all() and (V[:, IDX["g4_4"]] == 0).all()


def test_vertex_planted_mistake_is_caught():
    # forgetting the subsets in which v is isolated (here: a triangle seen from
    # an outside vertex) breaks the sum rule
    g = graphgen.from_edges(6, [(0, 1), (1, 2), (0, 2), (3, 4)])
    V = oracle.vertex_bruteforce(g)
    counts = oracle.bruteforce(g)
    assert int(V[:, IDX["g4_7"]].sum()) == 4 * counts[IDX["g4_7"]]
    V[3:, IDX["g4_7"]] = 0
    assert int(V[:, IDX["g4_7"]].sum()) != 4 * counts[IDX["g4_7"]]
