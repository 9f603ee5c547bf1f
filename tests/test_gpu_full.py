"""GPU parity at the benchmark sizes.

n = 4096 (directed, 95% density): every update kind, each checked in full
against the GPU cold blocked Floyd-Warshall of the updated graph and on
sampled rows against the oracle's Dijkstra; the cold start is checked in full
against the oracle's Floyd-Warshall.

n = 16384 (undirected complete, the benchmark graph): the cold start on one
row of every 128-row band against the oracle's Dijkstra; a block of the benchmark's update
stream, led by the worst-case increase (selected by the oracle), each update
checked in full against the GPU cold start of the updated graph and on
sampled rows against the oracle (at two checkpoints, one row per 128-row
band).  The light-edge scopes the
benchmark uses to pick that edge are checked against the oracle too, and so
are the final graph's pair node sets on sampled pairs.
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


def gpu_cold_equal(g, undirected):
    """Warm matrix == GPU cold Floyd-Warshall of the graph's adjacency."""
    import torch
    from paper_2412_15122_amd.apsp import Graph
    A = g.matrix_device("A")
    D = g.matrix_device("D")
    h = Graph(A, undirected=undirected, capacity=max(1, A.shape[0]))
    ok = bool(torch.equal(D, h.matrix_device("D")))
    h.close()
    return ok


def check_rows(g, A, ids, rows, what):
    """Sampled rows of the warm matrix == the oracle's Dijkstra on A."""
    pos = [ids.index(r) for r in rows]
    ref = O.dijkstra_rows(A, pos, threads=THREADS)
    D = g.matrix_device("D")
    got = D[pos].cpu().numpy()
    assert np.array_equal(got, ref), what


def band_rows(rng, ids, band=128):
    """One id from every band of `band` consecutive live positions."""
    n = len(ids)
    return [ids[min(n - 1, b + int(rng.integers(band)))] for b in range(0, n, band)]


def test_directed_n4096_every_update_kind():
    from paper_2412_15122_amd.apsp import Graph
    wl = W.config2()
    n = wl.adj.shape[0]
    g = Graph(wl.adj, undirected=False, capacity=n + 8)
    log("cold start n=4096")
    D_ref = O.fw(wl.adj, threads=THREADS)
    assert np.array_equal(g.matrix(), D_ref)
    A, ids = wl.adj.copy(), list(range(n))
    rng = np.random.default_rng(4096)
    for upd in wl.updates:
        log("update", upd.kind)
        if upd.kind == W.ADD:
            nid = g.add_node(upd.w_out, upd.w_in)
            A, ids = O.apply_update(A, ids, "add", w_out=upd.w_out, w_in=upd.w_in)
            touched = [nid]
        elif upd.kind == W.REMOVE:
            g.remove_node(upd.u)
            A, ids = O.apply_update(A, ids, "remove", u=upd.u)
            touched = []
        else:
            g.update_edge(upd.u, upd.v, upd.w)
            A, ids = O.apply_update(A, ids, "edge", u=upd.u, v=upd.v, w=upd.w)
            touched = [upd.u, upd.v]
        assert gpu_cold_equal(g, False), upd.kind
        sample = touched + [ids[int(x)] for x in rng.integers(0, len(ids), size=6)]
        check_rows(g, A, ids, sample, upd.kind)
    g.sync()


def oracle_worst_edge(adj, cands):
    """The oracle's pick of the worst-case increase: among the candidate
    edges, the largest |R| * |C| (ties: lowest (u, v)); undirected, so the
    columns of D are its rows."""
    ends = sorted({x for (u, v, _) in cands for x in (u, v)})
    rows = O.dijkstra_rows(adj, ends, threads=THREADS)
    at = {x: rows[i] for i, x in enumerate(ends)}
    scopes = {}
    for (u, v, w) in cands:
        scopes[(u, v)] = O.edge_scope(at[u], at[v], at[u], at[v], w)
    best = min(scopes, key=lambda e: (-(scopes[e][0] * scopes[e][1]), e))
    return best, scopes


def test_undirected_n16384_benchmark_stream():
    from paper_2412_15122_amd.apsp import Graph
    n = 16384
    adj = W.config3_graph(n)
    g = Graph(adj, undirected=True, capacity=n + 64)
    log("cold start n=16384")
    rng = np.random.default_rng(16384)
    ids = list(range(n))
    # one row in every 128-row band (the cold start's tile bands), at a seeded
    # offset, plus the first and last rows; undirected, so rows are columns too
    check_rows(g, adj, ids, band_rows(rng, ids) + [0, n - 1], "cold")

    cands = W.lightest_edges(adj, 64, True)
    (wu, wv), scopes = oracle_worst_edge(adj, cands)
    for (u, v, _) in cands:
        assert g.edge_scope(u, v) == scopes[(u, v)], (u, v)
    log("worst-case edge", wu, wv, scopes[(wu, wv)])

    stream = W.Config3Stream(adj, counts={W.ADD: 9, W.REMOVE: 6, W.DECREASE: 7, W.INCREASE: 8})
    block = stream.next_block(worst=(wu, wv, 20000))
    A = adj
    for t, upd in enumerate(block):
        log("update", t, upd.kind)
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
            touched = [upd.u, upd.v]
        if t == 0:
            s = g.stats()
            assert s["kind"] == 4 and s["flagged"] > 0  # the worst-case edge was tight
        assert gpu_cold_equal(g, True), (t, upd.kind)
        if t in (len(block) // 2, len(block) - 1):
            # checkpoints: one row per 128-row band of the live order
            check_rows(g, A, ids, touched + band_rows(rng, ids), f"checkpoint {t} {upd.kind}")
        elif t % 10 == 0 or upd.kind == W.REMOVE:
            sample = touched + [ids[int(x)] for x in rng.integers(0, len(ids), size=4)]
            check_rows(g, A, ids, sample, f"update {t} {upd.kind}")
    g.sync()
    # the final graph's pair node sets (Algorithms 8 and 10) on sampled pairs:
    # the oracle needs row i and column j only (undirected: column j = row j)
    for _ in range(4):
        a, b = (int(x) for x in rng.integers(0, len(ids), size=2))
        rows = O.dijkstra_rows(A, [a, b], threads=THREADS)
        on_o, key_o = O.pair_nodes_from(A, rows[0], rows[1], a, b)
        dist, on, key = g.query_nodes(ids[a], ids[b])
        assert dist == int(rows[0][b])
        assert on == [ids[p] for p in on_o] and key == [ids[p] for p in key_o], (a, b)
