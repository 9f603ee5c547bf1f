"""GPU parity of the serving loop (continuous batching over resident graphs).

A Poisson request stream over several graphs (edge increases and decreases,
node additions and removals, single-pair queries) is served under an HBM
budget that holds only a few graphs at once, so requests queue for
admission and idle graphs move out to host memory and back.  Each graph's
final matrix, ids and adjacency, each query answer and each new id must
equal what the same graph gets when its requests run alone, one library
call each, in arrival order.  Both schedules are covered: lockstep batches
of every request kind (with and without single calls at light load), and
the hybrid of work-queue batches and single calls.  A few final states are
also checked against the oracle's cold Floyd-Warshall.  The tolerance is
zero.
"""
import os

import numpy as np
import pytest

from oracle import oracle as O
from paper_2412_15122_amd import workloads as W

pytestmark = pytest.mark.gpu

THREADS = min(16, os.cpu_count() or 1)
HEADROOM = 64


def log(*a):
    print(*a, flush=True)


def graphs_and_requests(sizes, rate, count, seed):
    from paper_2412_15122_amd import serve
    adjs = [W.random_graph(n, 1, 10000, seed=seed * 100 + i) for i, n in enumerate(sizes)]
    gen = W.Config5Requests(adjs, seed=seed)
    reqs = serve.requests_from_stream(gen, rate, count)
    return adjs, gen, reqs


def replay_alone(adjs, reqs, minimax=False):
    """Each graph on its own, its requests in arrival order through the
    single calls."""
    from paper_2412_15122_amd.apsp import Graph
    gs = [Graph(a, capacity=a.shape[0] + HEADROOM, minimax=minimax) for a in adjs]
    results = {}
    for r in sorted(reqs, key=lambda r: r.arrival):
        g = gs[r.graph]
        if r.kind == "add":
            results[r.rid] = g.add_node(r.args[0], r.args[1])
        elif r.kind == "remove":
            g.remove_node(r.args[0])
        elif r.kind == "query":
            results[r.rid] = g.query(r.args[0], r.args[1])
        else:
            g.update_edge(*r.args)
    return gs, results


def check_against_alone(srv, adjs, reqs, minimax=False):
    import torch
    alone, results = replay_alone(adjs, reqs, minimax)
    for i in range(len(adjs)):
        g = srv.graph(i)
        if g is None:       # never admitted: no request addressed it
            assert not any(r.graph == i for r in reqs)
            continue
        assert g.ids() == alone[i].ids(), i
        assert torch.equal(g.matrix_device("D"), alone[i].matrix_device("D")), i
        assert torch.equal(g.matrix_device("A"), alone[i].matrix_device("A")), i
        g.sync()
    for r in reqs:
        if r.kind == "add" or (r.kind == "query" and not minimax):
            assert r.result == results[r.rid], (r.rid, r.kind)
        elif r.kind == "query":     # minimax: a batch and a single call may pick different optimal paths
            assert r.result[0] == results[r.rid][0], r.rid
    if minimax:
        check_minimax_paths(adjs, reqs)
    for g in alone:
        g.close()


def check_minimax_paths(adjs, reqs):
    """Every served minimax path, by property on the oracle's graph at the
    time of the query (each graph's requests replayed in arrival order): it
    runs from i to j over existing edges without repeating a node, and its
    largest edge weight is the oracle's minimax distance."""
    state = [(a, list(range(a.shape[0]))) for a in adjs]
    checked = 0
    for r in sorted(reqs, key=lambda r: r.arrival):
        A, ids = state[r.graph]
        if r.kind == "add":
            state[r.graph] = O.apply_update(A, ids, "add", w_out=r.args[0], w_in=r.args[1])
        elif r.kind == "remove":
            state[r.graph] = O.apply_update(A, ids, "remove", u=r.args[0])
        elif r.kind == "query":
            a, b = ids.index(r.args[0]), ids.index(r.args[1])
            d = int(O.minimax_rows(A, [a])[0][b])
            dist, path = r.result
            assert dist == d, r.rid
            if d >= W.INF:
                assert path == [], r.rid
                continue
            pos = [ids.index(x) for x in path]
            assert pos[0] == a and pos[-1] == b and len(set(pos)) == len(pos), r.rid
            assert all(A[x, y] < W.INF for x, y in zip(pos, pos[1:])), r.rid
            assert max((int(A[x, y]) for x, y in zip(pos, pos[1:])), default=0) == d, r.rid
            checked += 1
        else:
            state[r.graph] = O.apply_update(A, ids, "edge", u=r.args[0], v=r.args[1], w=r.args[2])
    assert checked > 0


@pytest.mark.parametrize("schedule,small", [("lockstep", 0), ("lockstep", 8), ("hybrid", 0)])
def test_mix_equals_alone_under_tiny_budget(schedule, small):
    from paper_2412_15122_amd import serve
    sizes = [60, 200, 33, 150, 90, 250, 120, 75]
    adjs, gen, reqs = graphs_and_requests(sizes, rate=20000.0, count=700, seed=51)
    from paper_2412_15122_amd import _native as N
    nbytes = sorted(int(N.load().apsp_required_bytes(a.shape[0] + HEADROOM, 0)) for a in adjs)
    budget = nbytes[-1] + nbytes[-2] + nbytes[-3]        # about three graphs at a time
    log("schedule", schedule, "small_batch", small)
    srv = serve.Server(adjs, budget_bytes=budget, streams=3, schedule=schedule, small_batch=small)
    summary = srv.run(reqs)
    log("summary", summary, dict(srv.stats))
    assert all(r.done is not None for r in reqs)
    assert srv.stats["evictions"] > 0 and srv.stats["swap_ins"] > 0
    if small == 0:                  # every request goes through a batch
        assert srv.stats["batches"] > 0 and srv.stats["single"] == 0
    if schedule == "hybrid":
        assert srv.stats["heavy"] > 0
    # per-graph FIFO: completion times never decrease along a graph's arrivals
    for i in range(len(adjs)):
        done = [r.done for r in sorted(reqs, key=lambda r: r.arrival) if r.graph == i]
        assert all(a <= b for a, b in zip(done, done[1:])), i
    check_against_alone(srv, adjs, reqs)
    # the oracle on some final states (the generator's bookkeeping holds them)
    for i in (0, 2, 4):
        st = gen.states[i]
        A = st.dense()
        assert srv.graph(i).ids() == st.live
        assert np.array_equal(srv.graph(i).matrix(), O.fw(A, threads=THREADS)), i
    srv.close()


@pytest.mark.parametrize("schedule", ["lockstep", "hybrid"])
def test_mix_equals_alone_with_everything_resident_and_slow_arrivals(schedule):
    from paper_2412_15122_amd import serve
    sizes = [300, 140, 64, 500]
    adjs, gen, reqs = graphs_and_requests(sizes, rate=3000.0, count=300, seed=52)
    log("schedule", schedule)
    srv = serve.Server(adjs, streams=4, schedule=schedule)
    summary = srv.run(reqs)
    log("summary", summary, dict(srv.stats))
    assert srv.stats["evictions"] == 0
    if schedule == "lockstep":      # light load: single calls on the batch stream
        assert srv.stats["single"] > 0
    check_against_alone(srv, adjs, reqs)
    srv.close()


def test_plain_server_matches_too():
    from paper_2412_15122_amd import serve
    from paper_2412_15122_amd.apsp import Graph
    import torch
    sizes = [80, 130]
    adjs, gen, reqs = graphs_and_requests(sizes, rate=5000.0, count=120, seed=53)
    gs = [Graph(a, capacity=a.shape[0] + HEADROOM) for a in adjs]
    summary = serve.serve_plain(gs, reqs)
    log("plain", summary)
    alone, results = replay_alone(adjs, reqs)
    for i in range(2):
        assert torch.equal(gs[i].matrix_device("D"), alone[i].matrix_device("D"))
    for r in reqs:
        if r.kind in ("add", "query"):
            assert r.result == results[r.rid]


def test_minimax_graphs_served_equal_alone():
    """The server over minimax graphs (lockstep batches of the minimax
    kernels): matrices, ids and new ids equal the single calls exactly,
    query distances too, and every served path is a minimax path of the
    graph at its time (by property); final states equal the oracle's minimax
    matrices."""
    from paper_2412_15122_amd import serve
    sizes = [60, 200, 33, 150]
    adjs, gen, reqs = graphs_and_requests(sizes, rate=20000.0, count=300, seed=53)
    srv = serve.Server(adjs, streams=2, schedule="lockstep", small_batch=0, minimax=True)
    summary = srv.run(reqs)
    log("summary", summary, dict(srv.stats))
    assert srv.stats["batches"] > 0
    check_against_alone(srv, adjs, reqs, minimax=True)
    for i in range(len(sizes)):
        st = gen.states[i]
        assert srv.graph(i).ids() == st.live
        assert np.array_equal(srv.graph(i).matrix(), O.minimax_apsp(st.dense())), i
    srv.close()
