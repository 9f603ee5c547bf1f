"""GPU parity of minimax (bottleneck) graphs: the same single-graph calls over
the (min, max) semiring (APSP_MINIMAX).

Every state is compared bit for bit with the oracle's minimax Floyd-Warshall
of the updated adjacency: the cold start (sizes across several 128-wide
tiles with ragged tails, 1 node, zero weights, many ties), then sequences of
every update kind -- add, remove, edge decrease, tight and loose increase,
deletion -- on directed and undirected graphs, with the cost fallback, with
an index of 2 entries (exhaustive scans), and with heavy rows (ties: rows
with more than 32 flags).  Removal statistics equal the oracle's minimax
mask; queries return a simple path whose largest edge is the distance, and
pair node sets equal the oracle's; a batch of minimax graphs equals the
single calls.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2412_15122_amd import workloads as W

pytestmark = pytest.mark.gpu

INF = W.INF


def log(*a):
    print(*a, flush=True)


def check_query(g, A, ids, D, rng, count=12):
    n = len(ids)
    for _ in range(count):
        a, b = (int(x) for x in rng.integers(0, n, size=2))
        dist, path = g.query(ids[a], ids[b])
        assert dist == int(D[a, b]), (a, b)
        if D[a, b] >= INF:
            assert path == []
            continue
        pos = [ids.index(v) for v in path]
        assert pos[0] == a and pos[-1] == b and len(set(pos)) == len(pos)
        assert max((int(A[x, y]) for x, y in zip(pos, pos[1:])), default=0) == D[a, b]


@pytest.mark.parametrize("undirected", [False, True])
def test_minimax_cold(undirected):
    from paper_2412_15122_amd.apsp import Graph
    rng = np.random.default_rng(11 + undirected)
    for n, wmax, dens, zero in ((1, 5, 1.0, 0.0), (17, 3, 0.5, 0.2), (129, 10000, 1.0, 0.0),
                                (143, 4, 0.1, 0.1), (300, 50, 0.05, 0.0), (257, 10000, 0.02, 0.0)):
        log("minimax cold", n, wmax, dens, zero, undirected)
        A = W.random_graph(n, 1, wmax, undirected=undirected, density=dens, seed=int(rng.integers(1 << 30)),
                           zero_frac=zero)
        g = Graph(A, undirected=undirected, capacity=n + 5, minimax=True)
        D = O.minimax_apsp(A)
        assert np.array_equal(g.matrix(), D), n
        check_query(g, A, list(range(n)), D, rng)
        g.close()


@pytest.mark.parametrize("undirected", [False, True])
@pytest.mark.parametrize("setup", ["plain", "fallback", "tiny_index"])
def test_minimax_updates(undirected, setup):
    from paper_2412_15122_amd.apsp import Graph
    rng = np.random.default_rng(23 + undirected + 10 * ("plain", "fallback", "tiny_index").index(setup))
    n = 150
    wmax = 8 if setup != "plain" else 3000
    A0 = W.random_graph(n, 1, wmax, undirected=undirected, density=0.3, seed=int(rng.integers(1 << 30)))
    g = Graph(A0, undirected=undirected, capacity=n + 12, minimax=True)
    if setup == "fallback":
        g.set_fallback(1, 0.3)
    if setup == "tiny_index":
        g.set_index_limit(2)
    st = W.GraphState(A0, undirected)
    kinds = [W.REMOVE, W.ADD, W.DECREASE, W.INCREASE, W.REMOVE, W.INCREASE, W.ADD, W.DECREASE] * 3
    for t, kind in enumerate(kinds):
        D_before = O.minimax_apsp(st.dense())
        ids_before = list(st.live)
        if kind == W.INCREASE and t % 3 == 0:
            # a tight increase: raise an edge that is the minimax path between its ends
            Ab = st.dense()
            tight = np.argwhere((Ab == D_before) & (Ab < INF) & ~np.eye(len(ids_before), dtype=bool))
            a, b = (int(x) for x in tight[int(rng.integers(len(tight)))])
            w = int(Ab[a, b]) + int(rng.integers(1, 2 * wmax))
            u, v = ids_before[a], ids_before[b]
            st.set_weight(u, v, w)
            g.update_edge(u, v, w)
        elif kind == W.INCREASE and t % 5 == 1:
            a, b = (int(x) for x in rng.choice(len(ids_before), size=2, replace=False))
            u, v = ids_before[a], ids_before[b]
            st.set_weight(u, v, INF)                   # deletion
            g.update_edge(u, v, INF)
        else:
            up = W.make_update(rng, st, kind, wmin=1, wmax=wmax, inc_max=2 * wmax, density=0.3)
            if up.kind == W.ADD:
                g.add_node(up.w_out, None if undirected else up.w_in)
            elif up.kind == W.REMOVE:
                g.remove_node(up.u)
                k = ids_before.index(up.u)
                F = O.remove_mask(D_before, k, minimax=True)
                s = g.stats()
                phi, cost = O.remove_cost(F, len(ids_before))
                assert s["rows"] == phi and s["cost"] == pytest.approx(cost), t
                if setup == "fallback":
                    assert s["fallback"] == (cost > 0.3)
                if not s["fallback"]:
                    assert s["flagged"] == int(F.sum()), t
            else:
                g.update_edge(up.u, up.v, up.w)
        A = st.dense()
        D = O.minimax_apsp(A)
        assert g.ids() == st.live
        assert np.array_equal(g.matrix(), D), (t, kind)
    check_query(g, A, list(st.live), D, rng)
    g.close()


@pytest.mark.parametrize("undirected", [True, False])
def test_minimax_heavy_rows_and_clone(undirected):
    """Weights 1..2 on a sparse graph: huge ties.  Directed, removals flag
    rows with far more than 32 entries (the block-per-row pass of the mask
    route); undirected, they take the spanning-forest route.  A clone keeps
    the semiring."""
    from paper_2412_15122_amd.apsp import Graph
    rng = np.random.default_rng(5)
    n = 600
    A0 = W.random_graph(n, 1, 2, undirected=undirected, density=0.02, seed=8)
    g = Graph(A0, undirected=undirected, capacity=n + 2, minimax=True)
    c = g.clone()
    st = W.GraphState(A0, undirected)
    for t in range(3):
        up = W.make_update(rng, st, W.REMOVE, wmin=1, wmax=2, inc_max=4)
        g.remove_node(up.u)
        c.remove_node(up.u)
        s = g.stats()
        if undirected:
            assert s["route"] == 1 and s["heavy_rows"] == 0
        else:
            assert s["route"] == 0 and s["heavy_rows"] > 0
    D = O.minimax_apsp(st.dense())
    assert np.array_equal(g.matrix(), D)
    assert np.array_equal(c.matrix(), D)
    g.close()
    c.close()


@pytest.mark.parametrize("undirected", [False, True])
def test_minimax_pair_nodes_equal_oracle(undirected):
    """Node sets of minimax pairs (on some / on every optimal walk) against
    the oracle's, on graphs with many ties and zero weights, cold and after
    updates (ids out of slot order)."""
    from paper_2412_15122_amd.apsp import Graph
    rng = np.random.default_rng(41 + undirected)
    for n, wmax, dens, zero in ((9, 3, 0.5, 0.2), (90, 4, 0.08, 0.1), (200, 30, 0.03, 0.0), (143, 10000, 0.05, 0.0)):
        A = W.random_graph(n, 1, wmax, undirected=undirected, density=dens, seed=int(rng.integers(1 << 30)),
                           zero_frac=zero)
        g = Graph(A, undirected=undirected, capacity=n + 8, minimax=True)
        st = W.GraphState(A, undirected)
        for kind in (W.REMOVE, W.ADD):
            up = W.make_update(rng, st, kind, wmin=1, wmax=wmax, inc_max=2 * wmax, density=dens)
            if up.kind == W.ADD:
                g.add_node(up.w_out, None if undirected else up.w_in)
            else:
                g.remove_node(up.u)
        Ad = st.dense()
        D = O.minimax_apsp(Ad)
        ids = st.live
        assert g.ids() == ids
        m = len(ids)
        pairs = [(int(a), int(b)) for a, b in rng.integers(0, m, size=(20, 2))] + [(0, 0), (m - 1, 0)]
        for a, b in pairs:
            on_o, key_o = O.minimax_pair_nodes(Ad, D, a, b)
            dist, on, key = g.query_nodes(ids[a], ids[b])
            assert dist == int(D[a, b]), (n, a, b)
            assert on == [ids[p] for p in on_o] and key == [ids[p] for p in key_o], (n, a, b)
        g.close()


def test_minimax_rejects_mixed_batches():
    from paper_2412_15122_amd.apsp import Graph
    from paper_2412_15122_amd.batch import Batch
    from paper_2412_15122_amd._native import ApspError
    A = W.random_graph(20, 1, 9, seed=2)
    g = Graph(A, capacity=24, minimax=True)
    h = Graph(A, capacity=24)
    b = Batch(2, 4)
    with pytest.raises(ApspError):                 # one batch, one path kind
        b.run([g, h], [("edge", 0, 1, 2, 3), ("edge", 1, 1, 2, 3)])
    assert np.array_equal(g.matrix(), O.minimax_apsp(A))
    assert np.array_equal(h.matrix(), O.fw(A))
    b.close()
    g.close()
    h.close()


@pytest.mark.parametrize("config", [{"use_graph": False, "variant": 1}, {"use_graph": True, "variant": 3}])
def test_minimax_batch_equals_single_calls(config):
    """Minimax graphs in one batched launch (the kernels' minimax build):
    every graph's matrices and ids equal the one-call-per-update path on a
    clone, each final matrix equals the oracle's, and query distances equal
    the single calls' (the paths may differ: both are minimax paths)."""
    from paper_2412_15122_amd.apsp import Graph
    from paper_2412_15122_amd.batch import Batch
    import torch
    rng = np.random.default_rng(31 + config["variant"])
    sizes = [1, 3, 40, 143, 300, 129, 700]
    ga, states, per, snap = [], [], [], {}
    for gi, n in enumerate(sizes):
        und = gi % 2 == 1
        wmax = (6, 5000)[gi % 3 == 0]
        A = W.random_graph(n, 1, wmax, undirected=und, density=0.4, seed=900 + gi)
        ga.append(Graph(A, undirected=und, capacity=n + 8, minimax=True))
        st = W.GraphState(A, und)
        seq = []
        for t in range(6):
            kinds = [W.ADD] + ([W.REMOVE] if len(st.live) >= 1 else []) + \
                    ([W.DECREASE, W.INCREASE] if len(st.live) >= 2 else [])
            k = kinds[int(rng.integers(len(kinds)))]
            try:
                up = W.make_update(rng, st, k, wmin=1, wmax=wmax, inc_max=2 * wmax, density=0.4)
            except RuntimeError:
                up = W.make_update(rng, st, W.ADD, wmin=1, wmax=wmax, inc_max=2 * wmax, density=0.4)
            if up.kind == W.ADD:
                seq.append(("add", gi, up.w_out, up.w_in))
            elif up.kind == W.REMOVE:
                seq.append(("remove", gi, up.u))
            else:
                seq.append(("edge", gi, up.u, up.v, up.w))
            if len(st.live) >= 2 and t % 2 == 1:
                a, c = rng.choice(len(st.live), size=2, replace=False)
                seq.append(("query", gi, st.live[int(a)], st.live[int(c)]))
                snap[(gi, len(seq) - 1)] = (st.dense(), list(st.live))
        states.append(st)
        per.append(seq)
    items = [it for t in range(max(map(len, per))) for seq in per if t < len(seq) for it in [seq[t]]]
    gb = [g.clone() for g in ga]
    b = Batch(len(ga), len(items), **config)
    res = b.run(ga, items)
    b.status()
    torch.cuda.synchronize()
    answers = {}
    for t, it in enumerate(items):
        g = gb[it[1]]
        if it[0] == "add":
            g.add_node(it[2], None if g.undirected else it[3])
        elif it[0] == "remove":
            g.remove_node(it[2])
        elif it[0] == "edge":
            g.update_edge(it[2], it[3], it[4])
        else:
            answers[t] = g.query(it[2], it[3])[0]
    for gi in range(len(ga)):
        assert ga[gi].ids() == gb[gi].ids() == states[gi].live
        assert torch.equal(ga[gi].matrix_device("D"), gb[gi].matrix_device("D")), gi
        assert torch.equal(ga[gi].matrix_device("A"), gb[gi].matrix_device("A")), gi
        assert np.array_equal(ga[gi].matrix(), O.minimax_apsp(states[gi].dense())), gi
    for t, d in answers.items():
        assert res[t].get()[0] == d, t
    # every batched path, by property on the oracle's graph when it was asked
    at = {}
    for t, it in enumerate(items):
        k = at.get(it[1], 0)
        at[it[1]] = k + 1
        if it[0] != "query":
            continue
        A, ids = snap[(it[1], k)]
        a, c = ids.index(it[2]), ids.index(it[3])
        d = int(O.minimax_rows(A, [a])[0][c])
        dist, path = res[t].get()
        assert dist == d, t
        if d >= INF:
            assert path == [], t
            continue
        pos = [ids.index(x) for x in path]
        assert pos[0] == a and pos[-1] == c and len(set(pos)) == len(pos), t
        assert max((int(A[x, y]) for x, y in zip(pos, pos[1:])), default=0) == d, t
    b.close()
    for g in ga + gb:
        g.close()


def test_minimax_benchmark_graph_n16384():
    """The benchmark graph (undirected complete, n = 16384) over the minimax
    semiring with Algorithm 5's cost fallback (delta = 0.5), as the bench
    runs it: the cold start and a block of the update stream, each state
    checked on sampled rows against the oracle's minimax Dijkstra, and
    minimax path queries on the final graph."""
    from paper_2412_15122_amd.apsp import Graph
    n = 16384
    adj = W.config3_graph(n)
    g = Graph(adj, undirected=True, capacity=n + 16, minimax=True)
    g.set_fallback(1, 0.5)
    rng = np.random.default_rng(216)
    ids = list(range(n))

    def check(A, ids, extra, what):
        pos = [ids.index(x) for x in extra] + [int(x) for x in rng.integers(0, len(ids), size=2)]
        got = g.matrix_device("D")[pos].cpu().numpy()
        assert np.array_equal(got, O.minimax_rows(A, pos)), what

    check(adj, ids, [0, n - 1], "cold")
    stream = W.Config3Stream(adj, counts={W.ADD: 3, W.REMOVE: 2, W.DECREASE: 3, W.INCREASE: 2})
    A = adj
    for t, upd in enumerate(stream.next_block()):
        log("minimax n=16384 update", t, upd.kind)
        if upd.kind == W.ADD:
            g.add_node(upd.w_out)
            A, ids = O.apply_update(A, ids, "add", w_out=upd.w_out, undirected=True)
            touched = [ids[-1]]
        elif upd.kind == W.REMOVE:
            g.remove_node(upd.u)
            A, ids = O.apply_update(A, ids, "remove", u=upd.u, undirected=True)
            touched = []
        else:
            g.update_edge(upd.u, upd.v, upd.w)
            A, ids = O.apply_update(A, ids, "edge", u=upd.u, v=upd.v, w=upd.w, undirected=True)
            touched = [upd.u]
        if t % 2 == 0 or upd.kind == W.REMOVE:
            check(A, ids, touched, f"update {t} {upd.kind}")
    assert g.ids() == ids
    # pair node sets on sampled pairs: the set on optimal walks exactly; the
    # reported key nodes pass the oracle's test, and so do no sampled others
    for _ in range(2):
        a, b = (int(x) for x in rng.integers(0, len(ids), size=2))
        rows = O.minimax_rows(A, [a, b])
        d = int(rows[0][b])
        dist, on, key = g.query_nodes(ids[a], ids[b])
        on_o = [int(t) for t in np.nonzero(np.maximum(rows[0].astype(np.int64), rows[1]) == d)[0]] if a != b else [a]
        assert dist == d and on == [ids[p] for p in on_o], (a, b)
        for t in key:
            assert O.minimax_key_test(A, a, b, d, ids.index(t)), (a, b, t)
        others = [p for p in on_o if p not in (a, b) and ids[p] not in key]
        for p in [others[int(x)] for x in rng.integers(0, len(others), size=3)] if others else []:
            assert not O.minimax_key_test(A, a, b, d, p), (a, b, p)
    pos = [int(x) for x in rng.integers(0, len(ids), size=3)]
    rows = O.minimax_rows(A, pos)
    for r, a in enumerate(pos):
        b = int(rng.integers(0, len(ids)))
        dist, path = g.query(ids[a], ids[b])
        assert dist == int(rows[r][b])
        p = [ids.index(v) for v in path]
        assert p[0] == a and p[-1] == b and len(set(p)) == len(p)
        assert max((int(A[x, y]) for x, y in zip(p, p[1:])), default=0) == dist
    g.close()


@pytest.mark.parametrize("wmax,limit", [(10000, None), (6, None), (10000, 2)])
def test_minimax_removal_by_spanning_forest(wmax, limit):
    """Removals on undirected minimax graphs take the spanning-forest route
    when its certificate holds (route 1): every state equals the oracle's
    minimax Floyd-Warshall, the changed-pair count equals the oracle's
    refined set (Theorem 6), and the mask's |F| and Phi equal the oracle's.
    With a 2-entry index the certificate cannot cover the graph and the mask
    route runs instead (route 0), with the same results."""
    from paper_2412_15122_amd.apsp import Graph
    rng = np.random.default_rng(91 + wmax + (limit or 0))
    n = 420
    A = W.random_graph(n, 1, wmax, undirected=True, seed=int(rng.integers(1 << 30)))
    g = Graph(A, undirected=True, capacity=n + 4, minimax=True)
    if limit:
        g.set_index_limit(limit)
    ids = list(range(n))
    D = O.minimax_apsp(A)
    routes = []
    for t in range(10):
        k = ids[int(rng.integers(len(ids)))]
        a = ids.index(k)
        F = O.remove_mask(D, a, minimax=True)
        g.remove_node(k)
        s = g.stats()
        A, ids = O.apply_update(A, ids, "remove", u=k, undirected=True)
        D2 = O.minimax_apsp(A)
        assert np.array_equal(g.matrix(), D2), (t, k)
        keep = [x for x in range(len(ids) + 1) if x != a]
        changed = O.refined_set(D[np.ix_(keep, keep)], D2)
        assert s["changed"] == int(changed.sum()), (t, s["changed"], int(changed.sum()))
        assert s["rows_changed"] == int(changed.any(axis=1).sum()), t
        assert s["flagged"] == int(F.sum()) and s["rows"] == int(F.any(axis=1).sum()), t
        routes.append(s["route"])
        D = D2
    if limit:
        assert set(routes) == {0}, routes
    else:
        assert routes.count(1) >= 8, routes


@pytest.mark.parametrize("wmax,density", [(30, 0.05), (10000, 1.0)])
def test_minimax_tight_increase_by_spanning_forest(wmax, density):
    """Tight increases (and deletions) of edges on undirected minimax graphs
    take the spanning-forest route (route 1): the forest of the graph before
    the change, and only the pairs across the two pieces the raised edge
    separates in it (none when it is not a forest edge).  Every state equals
    the oracle's minimax Floyd-Warshall, the changed-pair count equals the
    oracle's refined set, and the mask's |F| and Phi equal the oracle's."""
    from paper_2412_15122_amd.apsp import Graph
    rng = np.random.default_rng(131 + wmax)
    n = 360
    A = W.random_graph(n, 1, wmax, undirected=True, density=density, seed=int(rng.integers(1 << 30)))
    g = Graph(A, undirected=True, capacity=n + 4, minimax=True)
    ids = list(range(n))
    D = O.minimax_apsp(A)
    routes, moved = [], 0
    for t in range(12):
        tight = np.argwhere((A == D) & (A < INF) & ~np.eye(n, dtype=bool))
        # every other step, a raise that moves some distance (the edge
        # separates two pieces of the forest), found by trying candidates
        for _ in range(12 if t % 2 else 1):
            u, v = (int(x) for x in tight[int(rng.integers(len(tight)))])
            w_new = INF if t % 4 == 3 else int(A[u, v]) + int(rng.integers(1, wmax + 1))
            A2, ids2 = O.apply_update(A, ids, "edge", u=u, v=v, w=w_new, undirected=True)
            D2 = O.minimax_apsp(A2)
            if not np.array_equal(D2, D):
                break
        F = O.edge_mask(D, u, v, int(A[u, v]), True, minimax=True)
        g.update_edge(u, v, w_new)
        s = g.stats()
        A, ids = A2, ids2
        assert np.array_equal(g.matrix(), D2), (t, u, v, w_new)
        changed = O.refined_set(D, D2)
        assert s["kind"] == 4, (t, s)
        assert s["changed"] == int(changed.sum()), (t, s["changed"], int(changed.sum()))
        assert s["rows_changed"] == int(changed.any(axis=1).sum()), t
        assert s["flagged"] == int(F.sum()) and s["rows"] == int(F.any(axis=1).sum()), t
        routes.append(s["route"])
        moved += int(changed.sum()) > 0
        D = D2
    assert routes.count(1) >= 10, routes
    assert moved >= 3, moved


def test_widest_removal_by_spanning_forest():
    """The same route on an undirected widest graph (stored as a minimax one)."""
    from paper_2412_15122_amd.apsp import Graph
    rng = np.random.default_rng(97)
    n = 300
    C = W.random_graph(n, 1, 500, undirected=True, density=0.3, seed=98)
    g = Graph(C, undirected=True, capacity=n, widest=True)
    ids = list(range(n))
    for t in range(6):
        k = ids[int(rng.integers(len(ids)))]
        g.remove_node(k)
        C, ids = O.apply_update(C, ids, "remove", u=k, undirected=True)
        assert g.stats()["route"] == 1, t
        assert np.array_equal(g.matrix(), O.widest_apsp(C)), t
