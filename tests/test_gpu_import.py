"""GPU parity of the warm start from a known distance matrix (apsp_import) and
of growing a graph's capacity (apsp_grow).

The paper's problem statement (Section 1) starts from a graph whose
all-pairs shortest-path matrix is already known; apsp_import takes that
matrix, here the oracle's, instead of running a cold start.  Every later
result must equal the oracle run cold on the updated graph, bit for bit.
A matrix that is not a distance matrix of the adjacency is refused: by the
O(n^2) checks (range, zero diagonal, no entry above its edge, symmetry when
undirected) and, in the exact mode, by a cold recompute.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2412_15122_amd import workloads as W

pytestmark = pytest.mark.gpu

INF = W.INF


def Graph():
    from paper_2412_15122_amd.apsp import Graph as G
    return G


def ApspError():
    from paper_2412_15122_amd._native import ApspError as E
    return E


def expect_equal(g, A, ids, what, minimax=False):
    assert g.ids() == ids, what
    D = O.minimax_apsp(A) if minimax else O.fw(A)
    got = g.matrix()
    if not np.array_equal(got, D):
        bad = np.argwhere(got != D)
        i, j = bad[0]
        raise AssertionError(f"{what}: {len(bad)} entries differ, first ({ids[i]},{ids[j]}): "
                             f"gpu {got[i, j]} oracle {D[i, j]}")
    Ad = A.copy()
    np.fill_diagonal(Ad, 0)
    assert np.array_equal(g.adjacency(), Ad), what


def mixed_updates(g, A, ids, rng, steps, undirected, wmax, cap, what, minimax=False):
    """Random updates against whatever ids the graph holds (not only 0..n-1).
    An added node takes one above the largest id the graph ever held (the
    oracle's bookkeeping names it max(live ids) + 1, so the name is moved)."""
    for step in range(steps):
        kind = ("add", "remove", "decrease", "increase")[int(rng.integers(4))]
        if kind == "remove" and len(ids) <= 3:
            kind = "add"
        if kind == "add" and len(ids) >= cap:
            kind = "remove"
        if kind in ("decrease", "increase") and len(ids) < 2:
            kind = "add"
        if kind == "add":
            n = len(ids)
            w_out = rng.integers(1, wmax + 1, size=n).astype(np.int32)
            w_in = w_out if undirected else rng.integers(1, wmax + 1, size=n).astype(np.int32)
            expect_id = g.next_id()
            nid = g.add_node(w_out, None if undirected else w_in)
            A, ids = O.apply_update(A, ids, "add", w_out=w_out, w_in=w_in, undirected=undirected)
            assert nid == expect_id and nid >= ids[-1], what
            ids[-1] = nid
        elif kind == "remove":
            k = ids[int(rng.integers(len(ids)))]
            g.remove_node(k)
            A, ids = O.apply_update(A, ids, "remove", u=k, undirected=undirected)
        else:
            a, b = rng.choice(len(ids), size=2, replace=False)
            old = int(A[a, b])
            if kind == "decrease":
                w = int(rng.integers(1, min(old, wmax) + 1))
            else:
                w = int(rng.integers(min(old, 2 * wmax), 2 * wmax + 1))
            g.update_edge(ids[a], ids[b], w)
            A, ids = O.apply_update(A, ids, "edge", u=ids[a], v=ids[b], w=w, undirected=undirected)
        expect_equal(g, A, ids, f"{what} step {step} {kind}", minimax)
    return A, ids


@pytest.mark.parametrize("undirected", [False, True])
@pytest.mark.parametrize("n,wmax,density", [(0, 10, 1.0), (1, 10, 1.0), (130, 1000, 1.0), (257, 5, 0.6)])
@pytest.mark.parametrize("exact", [False, True])
def test_import_then_updates(n, wmax, density, undirected, exact):
    rng = np.random.default_rng(7 * n + 2 * undirected + exact)
    adj = W.random_graph(n, 1, wmax, undirected=undirected, density=density, seed=int(rng.integers(1 << 30)))
    D = O.fw(adj)
    g = Graph().from_matrix(adj, D, undirected=undirected, capacity=n + 6, exact=exact)
    ids = list(range(n))
    expect_equal(g, adj, ids, "import")
    mixed_updates(g, adj.copy(), ids, rng, 10, undirected, wmax, n + 6, f"n={n}")
    g.sync()


def test_import_keeps_given_ids():
    rng = np.random.default_rng(11)
    n = 200
    adj = W.random_graph(n, 1, 100, undirected=False, density=0.9, seed=5)
    ids = sorted(int(x) for x in rng.choice(100000, size=n, replace=False))
    g = Graph().from_matrix(adj, O.fw(adj), capacity=n + 4, ids=ids)
    expect_equal(g, adj, ids, "import with ids")
    i, j = ids[3], ids[150]
    d, path = g.query(i, j)
    a, b = ids.index(i), ids.index(j)
    assert d == O.fw(adj)[a, b]
    assert path == [ids[t] for t in O.canonical_path(adj, O.fw(adj), a, b)]
    mixed_updates(g, adj.copy(), ids, rng, 12, False, 100, n + 4, "ids")
    g.sync()


def test_import_minimax():
    rng = np.random.default_rng(3)
    n = 190
    adj = W.random_graph(n, 1, 50, undirected=True, density=0.8, seed=9)
    D = O.minimax_apsp(adj)
    g = Graph().from_matrix(adj, D, undirected=True, capacity=n + 4, minimax=True, exact=True)
    expect_equal(g, adj, list(range(n)), "minimax import", minimax=True)
    mixed_updates(g, adj.copy(), list(range(n)), rng, 8, True, 50, n + 4, "minimax", minimax=True)
    g.sync()


@pytest.mark.parametrize("undirected", [False, True])
def test_import_refuses_what_is_not_a_distance_matrix(undirected):
    n = 140
    adj = W.random_graph(n, 1, 1000, undirected=undirected, density=1.0, seed=21 + undirected)
    D = O.fw(adj)
    G, E = Graph(), ApspError()
    # an entry above its edge's weight
    i, j = np.argwhere((adj < INF) & ~np.eye(n, dtype=bool))[5]
    bad = D.copy()
    bad[i, j] = adj[i, j] + 1
    if undirected:
        bad[j, i] = bad[i, j]
    with pytest.raises(E):
        G.from_matrix(adj, bad, undirected=undirected, capacity=n)
    # a non-zero diagonal entry
    bad = D.copy()
    bad[7, 7] = 1
    with pytest.raises(E):
        G.from_matrix(adj, bad, undirected=undirected, capacity=n)
    # an entry outside [0, INF]
    bad = D.copy()
    bad[2, 9] = -4
    if undirected:
        bad[9, 2] = -4
    with pytest.raises(E):
        G.from_matrix(adj, bad, undirected=undirected, capacity=n)
    if undirected:
        bad = D.copy()
        bad[3, 4] -= 1          # still <= the edge, but no longer symmetric
        with pytest.raises(E):
            G.from_matrix(adj, bad, undirected=True, capacity=n)
    # one entry too small: passes the O(n^2) checks, refused by the exact mode
    strict = np.argwhere((D > 0) & (D < INF))
    a, b = strict[len(strict) // 2]
    bad = D.copy()
    bad[a, b] -= 1
    if undirected:
        bad[b, a] -= 1
    G.from_matrix(adj, bad, undirected=undirected, capacity=n).close()
    with pytest.raises(E):
        G.from_matrix(adj, bad, undirected=undirected, capacity=n, exact=True)
    # and the true matrix passes both
    g = G.from_matrix(adj, D, undirected=undirected, capacity=n, exact=True)
    expect_equal(g, adj, list(range(n)), "after refusals")
    g.sync()


@pytest.mark.parametrize("undirected", [False, True])
def test_grow_keeps_ids_and_distances(undirected):
    rng = np.random.default_rng(41 + undirected)
    n = 160
    adj = W.random_graph(n, 1, 500, undirected=undirected, density=1.0, seed=int(rng.integers(1 << 30)))
    g = Graph()(adj, undirected=undirected, capacity=n)
    A, ids = mixed_updates(g, adj.copy(), list(range(n)), rng, 6, undirected, 500, n, "before grow")
    while len(ids) < g.capacity:
        m = len(ids)
        w = rng.integers(1, 501, size=m).astype(np.int32)
        w_in = w if undirected else rng.integers(1, 501, size=m).astype(np.int32)
        nid = g.add_node(w, None if undirected else w_in)
        A, ids = O.apply_update(A, ids, "add", w_out=w, w_in=w_in, undirected=undirected)
        ids[-1] = nid
    with pytest.raises(ApspError()):       # full
        g.add_node(np.ones(len(ids), np.int32), None if undirected else np.ones(len(ids), np.int32))
    g.remove_node(ids[-1])                 # the largest id leaves: no copy may hand it out again
    A, ids = O.apply_update(A, ids, "remove", u=ids[-1], undirected=undirected)
    with pytest.raises(ApspError()):       # fewer slots than the graph uses
        g.grow(n - 1)
    big = g.grow(n + 40)
    assert big.capacity == n + 40
    assert big.next_id() == g.next_id() > max(ids) + 1
    expect_equal(big, A, ids, "grown")
    expect_equal(g, A, ids, "source unchanged")
    # the same copy by way of the import of its matrices
    imp = Graph().from_matrix(g.adjacency(), g.matrix(), undirected=undirected, capacity=n + 40, ids=ids,
                              next_id=g.next_id(), exact=True)
    assert imp.next_id() == big.next_id()
    A2, ids2 = A.copy(), list(ids)
    state = rng.bit_generator.state
    A, ids = mixed_updates(big, A, ids, rng, 14, undirected, 500, n + 40, "after grow")
    rng.bit_generator.state = state
    A2, ids2 = mixed_updates(imp, A2, ids2, rng, 14, undirected, 500, n + 40, "after import")
    assert ids2 == ids and np.array_equal(big.matrix(), imp.matrix())
    big.sync()
    imp.sync()
