"""Serving loop on the GPU: results identical alone and in the mix, budget
respected, failures isolated to their own request."""
import numpy as np
import pytest

import graphgen
import graphgen.configs as C
import oracle
import paper_1506_04322_amd as gl

pytestmark = pytest.mark.gpu


def dev(a):
    import torch

    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def standalone(g):
    return gl.graphlet_count(dev(g.row_ptr), dev(g.col), g.n)


def mixed_graphs(count, seed, m_max=200_000):
    reqs = C.serve_requests(count, seed=seed)
    out = []
    for _, kind, n, m, gseed in reqs:
        m = min(m, m_max)
        out.append(C.serve_graph(kind, max(16, 2 * m // 10), m, gseed))
    return out


def test_results_same_alone_and_in_the_mix():
    graphs = mixed_graphs(24, 101)
    with gl.Server(budget_bytes=32 << 30, slots=4) as srv:
        ids = [srv.submit(g.n, g.row_ptr, g.col) for g in graphs]
        results = [srv.wait(i) for i in ids]
        st = srv.stats()
    assert st["completed"] == len(graphs) and st["failed"] == 0
    for g, (counts, lat) in zip(graphs, results):
        assert counts == standalone(g)
        assert lat > 0
    for g, (counts, _) in list(zip(graphs, results))[:6]:
        assert counts == oracle.identity_route(g)


def small_graphs(count, seed):
    """Graphs of at most 1024 vertices (the batch lane's), of mixed sizes and
    densities, ER and torus random geometric."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        n = int(rng.integers(3, 1025))
        if i % 5 == 4:
            out.append(graphgen.rgg_torus(n, 8.0, int(rng.integers(1, 1 << 30))))
        else:
            m = int(rng.uniform(0.01, 0.3) * n * (n - 1) / 2)
            out.append(graphgen.er_gnm(n, max(m, 1), int(rng.integers(1, 1 << 30))))
    return out


def test_small_graphs_batched_same_alone_and_in_the_mix():
    # small graphs go to the batch lane, the others to the slots; every
    # result equals the standalone single-graph call and the oracle
    small = small_graphs(60, 505)
    big = mixed_graphs(8, 506, m_max=300_000)
    big = [g for g in big if g.n > gl.BATCH_MAX_N]
    order = small[:20] + big + small[20:]
    with gl.Server(budget_bytes=32 << 30, slots=4) as srv:
        ids = [srv.submit(g.n, g.row_ptr, g.col) for g in order]
        res = [srv.wait(i)[0] for i in ids]
        st = srv.stats()
    assert st["completed"] == len(order) and st["failed"] == 0
    assert st["batches"] >= 1 and st["batched"] == len(small)
    for g, counts in zip(order, res):
        assert counts == standalone(g)
    for g, counts in zip(order, res):
        if g.n <= gl.BATCH_MAX_N:
            assert counts == oracle.identity_route(g)


def test_failed_batch_isolates_its_request():
    # an asymmetric small graph in a burst of small graphs: under validation
    # its batch fails and is counted again one request at a time, so only it
    # fails
    good = small_graphs(40, 507)
    with gl.Server(budget_bytes=1 << 30, slots=2, validate=True) as srv:
        ids = [srv.submit(g.n, g.row_ptr, g.col) for g in good[:20]]
        bad = srv.submit(3, np.array([0, 1, 1, 2], np.int32), np.array([1, 0], np.int32))
        ids += [srv.submit(g.n, g.row_ptr, g.col) for g in good[20:]]
        with pytest.raises(gl.GraphletError) as e:
            srv.wait(bad)
        assert e.value.code == -4
        for g, i in zip(good, ids):
            assert srv.wait(i)[0] == standalone(g)
        st = srv.stats()
    assert st["failed"] == 1 and st["completed"] == len(good)


def test_admission_never_exceeds_budget():
    graphs = mixed_graphs(16, 202, m_max=400_000)
    # budget about two of the largest footprints: requests must queue
    big = max(graphs, key=lambda g: g.nnz)
    budget = None
    with gl.Server(budget_bytes=64 << 30, slots=1) as probe:
        rid = probe.submit(big.n, big.row_ptr, big.col)
        probe.wait(rid)
        budget = 2 * probe.stats()["bytes_peak"] + (1 << 20)
    import threading

    import torch

    # the device's own free memory, sampled while the requests run: what the
    # server holds never exceeds the budget (plus allocator rounding)
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    low = [free0]
    done = threading.Event()

    def sample():
        while not done.is_set():
            low[0] = min(low[0], torch.cuda.mem_get_info()[0])
            done.wait(0.0005)

    t = threading.Thread(target=sample)
    t.start()
    try:
        with gl.Server(budget_bytes=budget, slots=4) as srv:
            ids = [srv.submit(g.n, g.row_ptr, g.col) for g in graphs]
            res = [srv.wait(i) for i in ids]
            st = srv.stats()
    finally:
        done.set()
        t.join()
    assert st["bytes_peak"] <= budget
    assert free0 - low[0] <= budget + (64 << 20), (free0 - low[0], budget)
    assert st["completed"] == len(graphs)
    for g, (counts, _) in zip(graphs, res):
        assert counts == standalone(g)


def test_failures_are_isolated():
    good = graphgen.er_gnm(3000, 20000, 5)
    with gl.Server(budget_bytes=1 << 30, slots=2, validate=True) as srv:
        # malformed: a row pointing at an id out of range is refused at submit
        with pytest.raises(gl.GraphletError) as e:
            srv.submit(3, np.array([0, 1, 2, 2], np.int32), np.array([7, 0], np.int32))
        assert e.value.code == -1
        # asymmetric: passes the host checks, rejected by device validation
        bad = srv.submit(3, np.array([0, 1, 1, 2], np.int32), np.array([1, 0], np.int32))
        ok = srv.submit(good.n, good.row_ptr, good.col)
        with pytest.raises(gl.GraphletError) as e:
            srv.wait(bad)
        assert e.value.code == -4
        counts, _ = srv.wait(ok)
        assert counts == standalone(good)
    # a graph larger than the whole budget is rejected, the server stays up
    big = graphgen.er_gnm(200_000, 1_000_000, 6)  # CSR alone is 8.8 MB
    with gl.Server(budget_bytes=4 << 20, slots=1) as srv:
        with pytest.raises(gl.GraphletError) as e:
            srv.submit(big.n, big.row_ptr, big.col)
        assert e.value.code == -6
        tiny = graphgen.er_gnm(50, 100, 1)
        counts, _ = srv.wait(srv.submit(tiny.n, tiny.row_ptr, tiny.col))
        assert counts == oracle.bruteforce(tiny)


def test_cancel_pending_request():
    graphs = mixed_graphs(6, 303, m_max=300_000)
    with gl.Server(budget_bytes=32 << 30, slots=1) as srv:
        ids = [srv.submit(g.n, g.row_ptr, g.col) for g in graphs]
        srv.cancel(ids[-1])
        for i in ids[:-1]:
            srv.wait(i)
        with pytest.raises(gl.GraphletError):
            srv.wait(ids[-1])
        st = srv.stats()
    assert st["cancelled"] >= 1 and st["completed"] == len(graphs) - 1


# ------------------------------------------------------------ resident graphs


def _edge_set(g):
    eu, ev = oracle.edges(g)
    return set(zip(eu.tolist(), ev.tolist()))


def test_resident_graph_update_chain_vs_oracle():
    # a chain of insertions and deletions against a graph the server keeps:
    # every result equals the oracle's counts of the changed graph
    rng = np.random.default_rng(404)
    n = 36
    iu = np.triu_indices(n, 1)
    mask = rng.random(len(iu[0])) < 0.25
    edges = set(zip(iu[0][mask].tolist(), iu[1][mask].tolist()))
    g = graphgen.from_edges(n, sorted(edges))
    with gl.Server(budget_bytes=4 << 30, slots=3) as srv:
        gid = srv.register(g.n, g.row_ptr, g.col)
        counts, _ = srv.wait(gid)
        assert counts == oracle.bruteforce(g)
        rids, wants = [], []
        for _ in range(30):
            a, b = sorted(int(x) for x in rng.choice(n, 2, replace=False))
            insert = (a, b) not in edges
            edges.symmetric_difference_update({(a, b)})
            rids.append(srv.update(gid, a, b, insert))
            wants.append(oracle.bruteforce(graphgen.from_edges(n, sorted(edges))))
        for rid, want in zip(rids, wants):
            assert srv.wait(rid)[0] == want
        assert srv.graph_counts(gid) == wants[-1]
        # the kept CSR is the changed graph: a plain request on it agrees
        final = graphgen.from_edges(n, sorted(edges))
        assert srv.wait(srv.submit(final.n, final.row_ptr, final.col))[0] == wants[-1]
        srv.unregister(gid)
        with pytest.raises(gl.GraphletError):
            srv.update(gid, 0, 1, True)


def test_resident_graphs_interleaved_with_requests():
    # two resident graphs (one skewed, with hubs) updated in an interleaved
    # stream beside plain requests; each graph's updates apply in order
    rng = np.random.default_rng(505)
    gs = [graphgen.chung_lu(3000, 2.1, 3.0, 20000, 12), graphgen.rmat(11, 8, 0.57, 0.19, 0.19, 4)]
    sets = [_edge_set(g) for g in gs]
    plain = [graphgen.from_edges(50, [(i, (i * 7 + 3) % 50) for i in range(50) if i != (i * 7 + 3) % 50])]
    with gl.Server(budget_bytes=16 << 30, slots=4) as srv:
        gids = [srv.register(g.n, g.row_ptr, g.col) for g in gs]
        chains = [[], []]
        deg = [np.diff(g.row_ptr) for g in gs]
        for step in range(24):
            k = step % 2
            g, es = gs[k], sets[k]
            if step % 3 == 0:  # an edge at the highest-degree vertex
                hub = int(np.argmax(deg[k]))
                other = int(rng.integers(g.n))
                if other == hub:
                    other = (hub + 1) % g.n
                a, b = min(hub, other), max(hub, other)
            else:
                a, b = sorted(int(x) for x in rng.choice(g.n, 2, replace=False))
            insert = (a, b) not in es
            es.symmetric_difference_update({(a, b)})
            chains[k].append(srv.update(gids[k], a, b, insert))
            if step % 6 == 0:
                srv.submit(plain[0].n, plain[0].row_ptr, plain[0].col)
        for k in range(2):
            last = [srv.wait(r)[0] for r in chains[k]][-1]
            final = graphgen.from_edges(gs[k].n, sorted(sets[k]))
            assert last == oracle.identity_route(final)
            assert srv.graph_counts(gids[k]) == last
        for gid in gids:
            srv.unregister(gid)
        assert srv.stats()["failed"] == 0


def test_resident_graph_failed_updates_leave_it_unchanged():
    g = graphgen.from_edges(30, [(0, 1), (1, 2), (2, 0), (3, 4)])
    with gl.Server(budget_bytes=2 << 30, slots=2) as srv:
        gid = srv.register(g.n, g.row_ptr, g.col)
        base, _ = srv.wait(gid)
        bad = srv.update(gid, 5, 6, False)  # not an edge
        dup = srv.update(gid, 0, 1, True)   # already an edge
        ok = srv.update(gid, 3, 4, False)
        with pytest.raises(gl.GraphletError):
            srv.wait(bad)
        with pytest.raises(gl.GraphletError):
            srv.wait(dup)
        after = srv.wait(ok)[0]
        assert after == oracle.bruteforce(graphgen.from_edges(30, [(0, 1), (1, 2), (2, 0)]))
        assert srv.graph_counts(gid) == after
        with pytest.raises(gl.GraphletError):
            srv.update(gid, 0, 30, True)  # endpoint out of range
        with pytest.raises(gl.GraphletError):
            srv.update(gid + 1000, 0, 1, True)  # unknown graph
        srv.unregister(gid)
    assert base == oracle.bruteforce(g)


def test_resident_graph_room_runs_out():
    # an empty graph has room for 512 edges; the next insertion fails and the
    # graph keeps its counts
    n = 40
    g = graphgen.from_edges(n, [])
    pairs = [(a, b) for a in range(n) for b in range(a + 1, n)][:513]
    with gl.Server(budget_bytes=2 << 30, slots=1) as srv:
        gid = srv.register(g.n, g.row_ptr, g.col)
        srv.wait(gid)
        rids = [srv.update(gid, a, b, True) for a, b in pairs]
        for rid in rids[:-1]:
            srv.wait(rid)
        with pytest.raises(gl.GraphletError) as e:
            srv.wait(rids[-1])
        assert e.value.code == -6
        assert srv.graph_counts(gid) == oracle.bruteforce(graphgen.from_edges(n, pairs[:-1]))
        srv.unregister(gid)


def test_cancelled_registration_cancels_its_updates():
    # one slot kept busy by a large request, so the registration is still
    # pending when it is cancelled
    big = C.serve_graph("cl", 200_000, 1_000_000, 9)
    g = graphgen.from_edges(20, [(0, 1), (1, 2)])
    with gl.Server(budget_bytes=8 << 30, slots=1) as srv:
        busy = srv.submit(big.n, big.row_ptr, big.col)
        gid = srv.register(g.n, g.row_ptr, g.col)
        upd = srv.update(gid, 2, 3, True)
        srv.cancel(gid)
        for rid in (gid, upd):
            with pytest.raises(gl.GraphletError):
                srv.wait(rid)
        with pytest.raises(gl.GraphletError):
            srv.update(gid, 3, 4, True)
        srv.wait(busy)
        srv.unregister(gid)
        assert srv.stats()["cancelled"] >= 2


def test_cancelled_update_is_applied_only_if_it_finished():
    # an update cancelled right after its submission ends either CANCELLED
    # (pending or running: the graph and its counts are as before) or DONE
    # (it finished first: the change is applied); never half of each
    g = graphgen.rmat(14, 16, 0.57, 0.19, 0.19, 8)
    d = g.degrees()
    hub = int(np.argmax(d))
    eu, ev = oracle.edges(g)
    sel = np.nonzero((eu == hub) | (ev == hub))[0][:12]
    with gl.Server(budget_bytes=8 << 30, slots=1) as srv:
        gid = srv.register(g.n, g.row_ptr, g.col)
        counts, _ = srv.wait(gid)
        outcomes = set()
        for k in sel:
            a, b = int(eu[k]), int(ev[k])
            rid = srv.update(gid, a, b, False)
            srv.cancel(rid)
            try:
                after, _ = srv.wait(rid)
                outcomes.add("done")
                assert srv.graph_counts(gid) == after
                counts = gl.graphlet_update_edge(dev(g.row_ptr), dev(g.col), g.n, a, b, False,
                                                 counts)
                assert after == counts
                g, _ = _toggle_edge(g, a, b)
            except gl.GraphletError:
                outcomes.add("cancelled")
                assert srv.graph_counts(gid) == counts
        # the kept graph is still consistent: one more update applies cleanly
        a, b = int(eu[sel[-1]]), int(ev[sel[-1]])
        present = b in set(g.col[g.row_ptr[a]:g.row_ptr[a + 1]].tolist())
        got, _ = srv.wait(srv.update(gid, a, b, not present))
        g2, _ = _toggle_edge(g, a, b)
        assert got == standalone(g2)
        srv.unregister(gid)
    assert outcomes


def _toggle_edge(g, a, b):
    eu, ev = oracle.edges(g)
    edges = set(zip(eu.tolist(), ev.tolist()))
    key = (min(a, b), max(a, b))
    present = key in edges
    (edges.discard if present else edges.add)(key)
    return graphgen.from_edges(g.n, sorted(edges)), not present


def serve_pool_oracle_counts(graphs):
    """The oracle's counts of the serving benchmark's pool of graphs, stored
    by tests/golden/make_golden.py."""
    import json
    import os

    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "configs.json")
    with open(path) as f:
        gd = json.load(f)["serve_pool"]["graphs"]
    assert len(gd) == len(graphs)
    for g, want in zip(graphs, gd):
        assert g.sha256() == want["sha256"] and g.m == want["m"]
    return [[int(x) for x in want["counts"]] for want in gd]


def test_serve_pool_every_result_vs_oracle():
    # the benchmark's 96 graphs (1e3 to 2e6 edges, Chung-Lu and ER), all
    # submitted at once through 4 slots so that they overlap on the device,
    # then again one at a time: every result equals the oracle's counts
    _, graphs = C.serve_pool()
    want = serve_pool_oracle_counts(graphs)
    for slots, burst in ((4, True), (1, False)):
        with gl.Server(budget_bytes=64 << 30, slots=slots) as srv:
            if burst:
                ids = [srv.submit(g.n, g.row_ptr, g.col) for g in graphs]
                got = [srv.wait(i)[0] for i in ids]
            else:
                got = [srv.wait(srv.submit(g.n, g.row_ptr, g.col))[0] for g in graphs]
            st = srv.stats()
        assert st["completed"] == len(graphs) and st["failed"] == 0
        for i, (a, b) in enumerate(zip(got, want)):
            assert a == b, (slots, i)
