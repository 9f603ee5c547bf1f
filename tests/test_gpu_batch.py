"""GPU parity of batched updates (one persistent launch over many graphs).

Every graph's state after its queued items equals the one-call-per-update
path on a clone of the same graph (D, adjacency and ids, bit-exact); the
query answers equal the single-call query at the same point of the queue;
every graph's final state is also checked against the oracle's cold
Floyd-Warshall of its final adjacency (the 8300-node graph on one row per
128-row band, by the oracle's Dijkstra).  Sizes are uneven and include tiny
graphs (1 node, empty after a removal), n <= 143 and n just above a
128-slot pitch.  A rejected batch changes no graph.
"""
import os

import numpy as np
import pytest

from oracle import oracle as O
from paper_2412_15122_amd import workloads as W

pytestmark = pytest.mark.gpu

INF = W.INF
THREADS = min(16, os.cpu_count() or 1)


def log(*a):
    print(*a, flush=True)


def make_case(sizes, undirected_every=0, seed=7, updates=8, queries=True):
    """Graphs and a queued item list (tuples for Batch.run) with the
    GraphState bookkeeping of each graph."""
    rng = np.random.default_rng(seed)
    graphs, states, items = [], [], []
    for gi, n in enumerate(sizes):
        und = bool(undirected_every) and gi % undirected_every == 0
        adj = W.random_graph(n, 1, 5000, undirected=und, seed=seed * 1000 + gi)
        graphs.append((adj, und))
        states.append(W.GraphState(adj, und))
    per_graph = []
    for gi, st in enumerate(states):
        seq = []
        for t in range(updates):
            live = len(st.live)
            kinds = [W.ADD]
            if live >= 1:
                kinds.append(W.REMOVE)
            if live >= 2:
                kinds += [W.DECREASE, W.INCREASE]
            k = kinds[int(rng.integers(0, len(kinds)))]
            if k in (W.DECREASE, W.INCREASE):
                try:
                    up = W.make_update(rng, st, k, wmin=1, wmax=5000, inc_max=10000)
                except RuntimeError:           # no edge left between live nodes
                    up = W.make_update(rng, st, W.ADD, wmin=1, wmax=5000, inc_max=10000)
            else:
                up = W.make_update(rng, st, k, wmin=1, wmax=5000, inc_max=10000)
            if up.kind == W.ADD:
                seq.append(("add", gi, up.w_out, up.w_in))
            elif up.kind == W.REMOVE:
                seq.append(("remove", gi, up.u))
            else:
                seq.append(("edge", gi, up.u, up.v, up.w))
            if queries and len(st.live) >= 2 and t % 3 == 1:
                a, b = rng.choice(len(st.live), size=2, replace=False)
                seq.append(("query", gi, st.live[int(a)], st.live[int(b)]))
        per_graph.append(seq)
    # interleave the graphs' queues (per-graph order is what counts)
    pos = [0] * len(per_graph)
    while any(pos[g] < len(per_graph[g]) for g in range(len(per_graph))):
        for g in range(len(per_graph)):
            if pos[g] < len(per_graph[g]):
                items.append(per_graph[g][pos[g]])
                pos[g] += 1
    return graphs, states, items


def final_adjacency(adj, items, undirected):
    """The oracle's adjacency and ids after one graph's queued items."""
    A, ids = adj, list(range(adj.shape[0]))
    for it in items:
        if it[0] == "add":
            A, ids = O.apply_update(A, ids, "add", w_out=it[2], w_in=it[2] if undirected else it[3],
                                    undirected=undirected)
        elif it[0] == "remove":
            A, ids = O.apply_update(A, ids, "remove", u=it[2], undirected=undirected)
        elif it[0] == "edge":
            A, ids = O.apply_update(A, ids, "edge", u=it[2], v=it[3], w=it[4], undirected=undirected)
    return A, ids


def build(graphs):
    from paper_2412_15122_amd.apsp import Graph
    out = []
    for adj, und in graphs:
        n = adj.shape[0]
        out.append(Graph(adj, undirected=und, capacity=n + 8))
    return out


def replay_single(gs, items):
    """The one-call-per-update path; returns query answers by item index."""
    answers = {}
    for t, it in enumerate(items):
        g = gs[it[1]]
        if it[0] == "add":
            g.add_node(it[2], None if g.undirected else it[3])
        elif it[0] == "remove":
            g.remove_node(it[2])
        elif it[0] == "edge":
            g.update_edge(it[2], it[3], it[4])
        else:
            answers[t] = g.query(it[2], it[3])
    return answers


def assert_same(ga, gb, what):
    import torch
    assert ga.ids() == gb.ids(), what
    assert torch.equal(ga.matrix_device("D"), gb.matrix_device("D")), what
    assert torch.equal(ga.matrix_device("A"), gb.matrix_device("A")), what


def run_and_compare(sizes, config, undirected_every=0, seed=7, check_oracle=True):
    from paper_2412_15122_amd.batch import Batch
    import torch
    graphs, states, items = make_case(sizes, undirected_every, seed)
    ga = build(graphs)
    gb = [g.clone() for g in ga]
    b = Batch(len(ga), len(items), **config)
    log("batch", config, "graphs", len(ga), "items", len(items))
    res = b.run(ga, items)
    b.status()
    torch.cuda.synchronize()
    answers = replay_single(gb, items)
    for gi in range(len(ga)):
        assert_same(ga[gi], gb[gi], f"graph {gi} n0={sizes[gi]}")
        ga[gi].sync()
    for t, ans in answers.items():
        assert res[t].get() == ans, f"query item {t}"
    if check_oracle:
        for gi, st in enumerate(states):
            A = st.dense()
            assert ga[gi].ids() == st.live
            assert np.array_equal(ga[gi].matrix(), O.fw(A, threads=THREADS)), f"oracle graph {gi}"
    b.close()
    for g in ga + gb:
        g.close()


SIZES = [1, 2, 3, 17, 64, 100, 143, 144, 129, 250, 400, 777, 1500, 130, 5, 300]


def test_batch_equals_single_calls_direct_launch():
    run_and_compare(SIZES, {"use_graph": False})


def test_batch_equals_single_calls_graph_replay_both_variants():
    run_and_compare(SIZES, {"use_graph": True, "variant": 1, "order": 0}, undirected_every=3, seed=11)
    run_and_compare(SIZES, {"use_graph": True, "variant": 0, "order": 1, "grid": 3}, undirected_every=2, seed=12)


def test_lockstep_schedule_equals_single_calls():
    run_and_compare(SIZES, {"use_graph": False, "variant": 2}, undirected_every=3, seed=13)
    run_and_compare(SIZES, {"use_graph": True, "variant": 3}, undirected_every=2, seed=14)
    run_and_compare(SIZES, {"use_graph": True, "variant": 4}, undirected_every=3, seed=16)


def test_lockstep_with_a_tiny_grid_and_uneven_queues():
    """Grid far below the chunk count (every work-group loops over chunks and
    graphs) and graphs whose queues end at different steps."""
    run_and_compare([700, 3, 1, 250, 143, 1200], {"use_graph": True, "variant": 2, "grid": 3}, seed=15)


@pytest.mark.parametrize("variant", [0, 3])
def test_replayed_graph_stays_correct_across_batches(variant):
    """The recorded launch is replayed for later batches with new items."""
    from paper_2412_15122_amd.batch import Batch
    import torch
    sizes = [40, 200, 143, 600]
    graphs, _, items1 = make_case(sizes, 0, seed=21)
    ga = build(graphs)
    gb = [g.clone() for g in ga]
    b = Batch(len(ga), 256, use_graph=True, variant=variant)
    for rnd in range(3):
        if rnd == 0:
            items = items1
        else:   # fresh edge updates and queries on the current ids
            rng = np.random.default_rng(100 + rnd)
            items = []
            for gi, g in enumerate(ga):
                ids = g.ids()
                for _ in range(5):
                    u, v = rng.choice(len(ids), size=2, replace=False)
                    items.append(("edge", gi, ids[int(u)], ids[int(v)], int(rng.integers(1, 12000))))
                a, c = rng.choice(len(ids), size=2, replace=False)
                items.append(("query", gi, ids[int(a)], ids[int(c)]))
        res = b.run(ga, items)
        b.status()
        torch.cuda.synchronize()
        answers = replay_single(gb, items)
        for gi in range(len(ga)):
            assert_same(ga[gi], gb[gi], f"round {rnd} graph {gi}")
        for t, ans in answers.items():
            assert res[t].get() == ans
    b.close()


def test_rejected_batch_changes_nothing():
    from paper_2412_15122_amd.batch import Batch
    from paper_2412_15122_amd._native import ApspError
    import torch
    sizes = [50, 90]
    graphs, _, items = make_case(sizes, 0, seed=31, queries=False)
    ga = build(graphs)
    before = [(g.ids(), g.matrix_device("D").clone(), g.matrix_device("A").clone()) for g in ga]
    bad = list(items)
    bad.insert(len(bad) // 2, ("edge", 1, 10 ** 6, 0, 5))  # 10**6 is not a live id
    b = Batch(2, len(bad), use_graph=True)
    with pytest.raises(ApspError):
        b.run(ga, bad)
    for g, (ids, D, A) in zip(ga, before):
        assert g.ids() == ids
        assert torch.equal(g.matrix_device("D"), D) and torch.equal(g.matrix_device("A"), A)
    # the same batch without the bad item then runs as usual
    gb = [g.clone() for g in ga]
    b.run(ga, items)
    torch.cuda.synchronize()
    replay_single(gb, items)
    for gi in range(2):
        assert_same(ga[gi], gb[gi], f"graph {gi}")
    b.close()


def test_large_batch_checked_on_host_threads():
    """From 512 items on, the host checks split the graphs over threads: a
    batch with bad items in two graphs is rejected naming the earlier one,
    with every graph unchanged, and the valid batch still equals the single
    calls and the oracle."""
    from paper_2412_15122_amd.batch import Batch
    from paper_2412_15122_amd._native import ApspError
    import torch
    sizes = [20 + (7 * i) % 41 for i in range(80)]
    graphs, states, items = make_case(sizes, undirected_every=4, seed=41)
    assert len(items) >= 512
    ga = build(graphs)
    before = [(g.ids(), g.matrix_device("D").clone(), g.matrix_device("A").clone()) for g in ga]
    bad = list(items)
    bad.insert(len(bad) * 3 // 4, ("edge", 70, 10 ** 6, 0, 5))  # 10**6 is not a live id
    early = len(bad) // 4
    bad.insert(early, ("remove", 5, 10 ** 6))
    b = Batch(len(ga), len(bad), use_graph=True, variant=3)
    with pytest.raises(ApspError, match=rf"item {early}: id is not live"):
        b.run(ga, bad)
    for g, (ids, D, A) in zip(ga, before):
        assert g.ids() == ids
        assert torch.equal(g.matrix_device("D"), D) and torch.equal(g.matrix_device("A"), A)
    gb = [g.clone() for g in ga]
    res = b.run(ga, items)
    b.status()
    torch.cuda.synchronize()
    answers = replay_single(gb, items)
    for gi in range(len(ga)):
        assert_same(ga[gi], gb[gi], f"graph {gi}")
    for t, ans in answers.items():
        assert res[t].get() == ans, f"query item {t}"
    for gi in (0, 1, 37, 79):
        assert ga[gi].ids() == states[gi].live
        assert np.array_equal(ga[gi].matrix(), O.fw(states[gi].dense(), threads=THREADS)), f"oracle graph {gi}"
    b.close()
    for g in ga + gb:
        g.close()


def test_config4_shape_sample():
    """A slice of the batched workload (directed complete graphs, n
    log-uniform in [128, 2048], 8 queued updates each)."""
    from paper_2412_15122_amd.batch import Batch
    import torch
    wls = W.config4(graphs=12)
    from paper_2412_15122_amd.apsp import Graph
    ga = [Graph(w.adj, undirected=False, capacity=w.adj.shape[0] + 8) for w in wls]
    gb = [g.clone() for g in ga]
    items = []
    for gi, w in enumerate(wls):
        for up in w.updates:
            if up.kind == W.ADD:
                items.append(("add", gi, up.w_out, up.w_in))
            elif up.kind == W.REMOVE:
                items.append(("remove", gi, up.u))
            else:
                items.append(("edge", gi, up.u, up.v, up.w))
    gc = [g.clone() for g in ga]
    for variant, gs in ((0, ga), (3, gc)):
        b = Batch(len(gs), len(items), variant=variant)
        b.run(gs, items)
        b.status()
        b.close()
    torch.cuda.synchronize()
    replay_single(gb, items)
    for gi in range(len(ga)):
        assert_same(ga[gi], gb[gi], f"graph {gi} n={wls[gi].adj.shape[0]}")
        assert_same(gc[gi], gb[gi], f"lockstep graph {gi} n={wls[gi].adj.shape[0]}")
        A, ids = final_adjacency(wls[gi].adj, [it for it in items if it[1] == gi], False)
        assert gc[gi].ids() == ids
        assert np.array_equal(gc[gi].matrix(), O.fw(A, threads=THREADS)), f"oracle graph {gi}"


def test_lockstep_large_pitch_heavy_rows_tiny_index():
    """A graph whose pitch exceeds 8192 columns (its heavy-row need bitmap is
    longer than the lockstep wave lists it shares LDS with), small weights
    (many ties: rows with more than 32 flags) and an index of 2 entries
    (recomputed entries above the bound take exhaustive scans), beside small
    graphs: the lockstep batch equals the single calls."""
    from paper_2412_15122_amd.apsp import Graph
    from paper_2412_15122_amd.batch import Batch
    import torch
    rng = np.random.default_rng(5)
    sizes = [8300, 40, 300]
    adjs = [W.random_graph(n, 1, 6, seed=500 + i) for i, n in enumerate(sizes)]
    ga = [Graph(a, capacity=a.shape[0] + 4) for a in adjs]
    for g in ga:
        g.set_index_limit(2)
    gb = [g.clone() for g in ga]
    items = []
    for gi, a in enumerate(adjs):
        n = a.shape[0]
        ones = np.argwhere(a == 1)
        ones = ones[ones[:, 0] != ones[:, 1]]
        removed = set()
        for t in range(3):
            u, v = (int(x) for x in ones[int(rng.integers(len(ones)))])
            if u not in removed and v not in removed:
                items.append(("edge", gi, u, v, 4))   # a weight-1 edge is tight: the increase masks
            k = int(rng.integers(n))
            while k in removed:
                k = int(rng.integers(n))
            removed.add(k)
            items.append(("remove", gi, k))
    b = Batch(len(ga), len(items), variant=3, use_graph=True)
    log("items", len(items))
    b.run(ga, items)
    b.status()
    torch.cuda.synchronize()
    replay_single(gb, items)
    for gi in range(len(ga)):
        assert_same(ga[gi], gb[gi], f"graph {gi} n0={sizes[gi]}")
        ga[gi].sync()
        A, ids = final_adjacency(adjs[gi], [it for it in items if it[1] == gi], False)
        assert ga[gi].ids() == ids
        if sizes[gi] <= 2048:
            assert np.array_equal(ga[gi].matrix(), O.fw(A, threads=THREADS)), f"oracle graph {gi}"
        else:
            pos = [min(len(ids) - 1, b + int(rng.integers(128))) for b in range(0, len(ids), 128)]
            ref = O.dijkstra_rows(A, pos, threads=THREADS)
            assert np.array_equal(ga[gi].matrix_device("D")[pos].cpu().numpy(), ref), f"oracle graph {gi}"
    b.close()
    for g in ga + gb:
        g.close()
