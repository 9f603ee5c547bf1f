"""GPU parity of apsp_query_nodes: the nodes on some and on every shortest
path of a pair (Algorithms 7, 8 and 10).

Both lists are compared exactly with the oracle's `pair_nodes` (candidate set
by its definition; key nodes by reachability with each candidate taken out),
on graphs with many ties (weights 1..3), with zero-weight edges (levels
joined inside: the device's in-level search runs), directed and undirected,
after warm updates (ids no longer in slot order), for i == j, unreachable
pairs, and a chain whose every interior node is a key node (more than 1024
candidates: several passes of the gather and emit loops).
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2412_15122_amd import workloads as W

pytestmark = pytest.mark.gpu

INF = W.INF


def log(*a):
    print(*a, flush=True)


def searched_levels(A, D, i, j):
    """Candidates (not i, j) on a level that holds other candidates and a
    zero-weight edge between two of its candidates: the cases that take the
    in-level search rather than the level count alone."""
    if i == j or D[i, j] >= INF:
        return 0
    d = int(D[i, j])
    on = [t for t in range(len(D)) if int(D[i, t]) + int(D[t, j]) == d]
    lev = {t: int(D[i, t]) for t in on}
    out = 0
    for t in on:
        if t in (i, j):
            continue
        same = [x for x in on if lev[x] == lev[t]]
        if len(same) > 1 and any(A[x, y] == 0 for x in same for y in same if x != y):
            out += 1
    return out


def check_pairs(g, A, ids, pairs, what):
    D = O.fw(A)
    pos = {v: p for p, v in enumerate(ids)}
    searched = 0
    for a, b in pairs:
        searched += searched_levels(A, D, a, b)
        dist, on, key = g.query_nodes(ids[a], ids[b])
        on_o, key_o = O.pair_nodes(A, D, a, b)
        assert dist == int(min(D[a, b], INF)), (what, a, b)
        assert on == [ids[p] for p in on_o], (what, a, b)
        assert key == [ids[p] for p in key_o], (what, a, b)
        assert all(pos[v] in on_o for v in key)
    return searched


@pytest.mark.parametrize("undirected", [False, True])
@pytest.mark.parametrize("zero", [0.0, 0.25])
def test_query_nodes_equal_oracle(undirected, zero):
    from paper_2412_15122_amd.apsp import Graph
    rng = np.random.default_rng(3 + undirected + int(100 * zero))
    searched = 0
    for n, wmax, dens in ((7, 3, 0.5), (90, 3, 0.15), (143, 2, 0.05), (60, 5, 0.3)):
        log("query_nodes", n, wmax, dens, undirected, zero)
        adj = W.random_graph(n, 1, wmax, undirected=undirected, density=dens,
                             seed=int(rng.integers(1 << 30)), zero_frac=zero)
        g = Graph(adj, undirected=undirected, capacity=n + 4)
        pairs = [(int(a), int(b)) for a, b in rng.integers(0, n, size=(40, 2))] + [(0, 0), (0, n - 1)]
        searched += check_pairs(g, adj, list(range(n)), pairs, f"cold n={n}")
        g.close()
    log("candidates decided by the in-level search:", searched)
    if zero:
        assert searched > 0


@pytest.mark.parametrize("undirected", [False, True])
def test_query_nodes_after_warm_updates(undirected):
    """Removals, additions (ids reuse freed slots: slot order is no longer id
    order) and edge changes, then queries on the current graph."""
    from paper_2412_15122_amd.apsp import Graph
    rng = np.random.default_rng(17 + undirected)
    n = 120
    adj = W.random_graph(n, 1, 3, undirected=undirected, density=0.08, seed=99 + undirected, zero_frac=0.1)
    g = Graph(adj, undirected=undirected, capacity=n + 8)
    st = W.GraphState(adj, undirected)
    for t in range(12):
        kind = (W.REMOVE, W.ADD, W.DECREASE, W.INCREASE)[t % 4]
        up = W.make_update(rng, st, kind, wmin=0, wmax=3, inc_max=6, density=0.1)
        if up.kind == W.ADD:
            g.add_node(up.w_out, None if undirected else up.w_in)
        elif up.kind == W.REMOVE:
            g.remove_node(up.u)
        else:
            g.update_edge(up.u, up.v, up.w)
    assert g.ids() == st.live
    A = st.dense()
    m = len(st.live)
    pairs = [(int(a), int(b)) for a, b in rng.integers(0, m, size=(40, 2))]
    pairs += [(m - 1, 0), (0, m - 1)]            # the newest node (a reused slot)
    check_pairs(g, A, st.live, pairs, "warm")
    g.close()


def test_query_nodes_unreachable_and_single():
    from paper_2412_15122_amd.apsp import Graph
    adj = np.full((5, 5), INF, dtype=np.int32)
    np.fill_diagonal(adj, 0)
    adj[0, 1] = adj[1, 2] = 4
    g = Graph(adj, capacity=8)
    assert g.query_nodes(0, 3) == (INF, [], [])
    assert g.query_nodes(2, 0) == (INF, [], [])
    assert g.query_nodes(4, 4) == (0, [4], [])
    assert g.query_nodes(0, 2) == (8, [0, 1, 2], [1])
    g.close()


def test_query_nodes_long_chain_and_capacity():
    """0 -> 1 -> ... -> n-1 (weight 1) plus longer bypasses: every interior
    node is a key node; a bypass of the same length as the stretch it skips
    takes the skipped nodes out of the key set."""
    from paper_2412_15122_amd.apsp import Graph
    from paper_2412_15122_amd._native import ApspError
    n = 1300
    adj = np.full((n, n), INF, dtype=np.int32)
    np.fill_diagonal(adj, 0)
    for t in range(n - 1):
        adj[t, t + 1] = 1
    adj[10, 20] = 11                              # longer than the 10 steps it skips
    adj[500, 503] = 3                             # as long: 501, 502 are no longer key nodes
    g = Graph(adj, capacity=n + 3)
    dist, on, key = g.query_nodes(0, n - 1)
    assert dist == n - 1
    assert on == list(range(n))
    assert key == [t for t in range(1, n - 1) if t not in (501, 502)]
    dist, on, key = g.query_nodes(400, 900)
    assert (dist, on) == (500, list(range(400, 901)))
    assert key == [t for t in range(401, 900) if t not in (501, 502)]
    # buffers too small: APSP_E_CAPACITY
    import ctypes
    from paper_2412_15122_amd import _native as N
    d, a, b = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    buf = (ctypes.c_int32 * 4)()
    st = g._lib.apsp_query_nodes(g._h, 0, n - 1, ctypes.byref(d), buf, 4, ctypes.byref(a), buf, 4, ctypes.byref(b))
    assert st == N.APSP_E_CAPACITY and a.value == n and b.value == n - 4 and d.value == n - 1
    with pytest.raises(ApspError):
        g.query_nodes(0, n + 5)
    g.close()


@pytest.mark.parametrize("undirected", [False, True])
def test_query_paths_are_algorithm_8s_list(undirected):
    """Graph.query_paths: every listed path is a shortest path (its length
    is D[i][j]); with positive weights its node sets cover the candidate
    set, and the nodes on every listed path include the key nodes."""
    from paper_2412_15122_amd.apsp import Graph
    rng = np.random.default_rng(77 + undirected)
    n = 80
    A = W.random_graph(n, 1, 3, undirected=undirected, density=0.12, seed=5 + undirected)
    g = Graph(A, undirected=undirected, capacity=n)
    D = O.fw(A)
    for _ in range(25):
        a, b = (int(x) for x in rng.integers(0, n, size=2))
        paths = g.query_paths(a, b)
        on, key = O.pair_nodes(A, D, a, b)
        if a == b:
            assert paths == [[a]]
            continue
        if D[a, b] >= INF:
            assert paths == []
            continue
        for p in paths:
            assert p[0] == a and p[-1] == b
            assert sum(int(A[x, y]) for x, y in zip(p, p[1:])) == D[a, b]
        assert sorted(set().union(*map(set, paths))) == on
        common = set.intersection(*map(set, paths)) - {a, b}
        assert set(key) <= common
    g.close()


@pytest.mark.parametrize("undirected", [False, True])
def test_query_nodes_mostly_zero_weights(undirected):
    """Weights mostly 0 (zero-weight cycles, levels holding most candidates,
    the in-level search for nearly every candidate)."""
    from paper_2412_15122_amd.apsp import Graph
    rng = np.random.default_rng(123 + undirected)
    n = 120
    A = W.random_graph(n, 1, 2, undirected=undirected, density=0.06, seed=31 + undirected, zero_frac=0.7)
    g = Graph(A, undirected=undirected, capacity=n)
    D = O.fw(A)
    pairs = [(int(a), int(b)) for a, b in rng.integers(0, n, size=(6, 2))]
    searched = check_pairs(g, A, list(range(n)), pairs, "zero-heavy")
    log("candidates decided by the in-level search:", searched)
    g.close()
