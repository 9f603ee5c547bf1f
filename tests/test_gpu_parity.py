"""GPU parity: every result of the HIP library equals the CPU oracle run cold on
the updated graph, bit for bit (integer arithmetic: the bar is equality).

Sizes are small enough for the oracle to finish in seconds while spanning
several 128-wide tiles and ragged tails.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2412_15122_amd import workloads as W

pytestmark = pytest.mark.gpu

INF = W.INF


def lib_graph(adj, undirected, capacity=None):
    from paper_2412_15122_amd.apsp import Graph
    return Graph(adj, undirected=undirected, capacity=capacity)


def expect_equal(g, A, ids, what=""):
    assert g.ids() == ids, what
    D = O.fw(A)
    got = g.matrix()
    if not np.array_equal(got, D):
        bad = np.argwhere(got != D)
        i, j = bad[0]
        raise AssertionError(f"{what}: {len(bad)} entries differ, first ({ids[i]},{ids[j]}): "
                             f"gpu {got[i, j]} oracle {D[i, j]}")
    Ad = A.copy()
    np.fill_diagonal(Ad, 0)
    assert np.array_equal(g.adjacency(), Ad), what
    return D


def apply(g, A, ids, upd, undirected):
    if upd.kind == W.ADD:
        nid = g.add_node(upd.w_out, upd.w_in)
        A, ids = O.apply_update(A, ids, "add", w_out=upd.w_out, w_in=upd.w_in, undirected=undirected)
        assert nid == ids[-1]
    elif upd.kind == W.REMOVE:
        g.remove_node(upd.u)
        A, ids = O.apply_update(A, ids, "remove", u=upd.u, undirected=undirected)
    else:
        g.update_edge(upd.u, upd.v, upd.w)
        A, ids = O.apply_update(A, ids, "edge", u=upd.u, v=upd.v, w=upd.w, undirected=undirected)
    return A, ids


# ---------------------------------------------------------------------------
# cold start
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("undirected", [False, True])
@pytest.mark.parametrize("n", [0, 1, 2, 5, 127, 128, 129, 300, 513])
def test_cold_matches_oracle(n, undirected):
    rng = np.random.default_rng(n * 7 + undirected)
    for density, wmax, zero in ((1.0, 1000, 0.0), (0.3, 3, 0.0), (0.05, 100, 0.2)):
        adj = W.random_graph(n, 1, wmax, undirected=undirected, density=density,
                             seed=int(rng.integers(1 << 30)), zero_frac=zero)
        g = lib_graph(adj, undirected, capacity=max(n, 1) + 3)
        expect_equal(g, adj, list(range(n)), f"cold n={n}")
        g.sync()


# ---------------------------------------------------------------------------
# the small workload: one update of each kind
# ---------------------------------------------------------------------------

def test_config1_sequence():
    wl = W.config1()
    g = lib_graph(wl.adj, False, capacity=300)
    A, ids = wl.adj.copy(), list(range(256))
    expect_equal(g, A, ids, "cold")
    for upd in wl.updates:
        A, ids = apply(g, A, ids, upd, False)
        expect_equal(g, A, ids, upd.kind)
    g.sync()


# ---------------------------------------------------------------------------
# random update sequences
# ---------------------------------------------------------------------------

def random_sequence(seed, n, undirected, steps, wmax, density=1.0, zero=0.0, limit=None, cap_extra=12,
                    inf_edges=False):
    rng = np.random.default_rng(seed)
    adj = W.random_graph(n, 1, wmax, undirected=undirected, density=density,
                         seed=int(rng.integers(1 << 30)), zero_frac=zero)
    g = lib_graph(adj, undirected, capacity=n + cap_extra)
    if limit:
        g.set_index_limit(limit)
    st = W.GraphState(adj, undirected)
    A, ids = adj.copy(), list(range(n))
    expect_equal(g, A, ids, "cold")
    for step in range(steps):
        kinds = [W.ADD, W.REMOVE, W.DECREASE, W.INCREASE] + ([W.DELETE, W.INSERT] * 2 if inf_edges else [])
        kind = kinds[int(rng.integers(len(kinds)))]
        if len(st.live) <= 2 and kind == W.REMOVE:
            kind = W.ADD
        if len(ids) >= n + cap_extra and kind == W.ADD:
            kind = W.REMOVE
        upd = W.make_update(rng, st, kind, wmin=1, wmax=wmax, inc_max=2 * wmax, density=density)
        A, ids = apply(g, A, ids, upd, undirected)
        expect_equal(g, A, ids, f"step {step} {kind}")
    g.sync()


@pytest.mark.parametrize("undirected", [False, True])
@pytest.mark.parametrize("n,wmax,density", [(40, 20, 1.0), (150, 1000, 1.0), (200, 5, 0.5), (331, 10000, 0.95)])
def test_random_sequences(n, wmax, density, undirected):
    random_sequence(1000 + n + undirected, n, undirected, 14, wmax, density)


@pytest.mark.parametrize("undirected", [False, True])
@pytest.mark.parametrize("density", [0.95, 0.5])
def test_random_sequences_delete_and_insert_edges(density, undirected):
    """Edge updates that cross INF: an existing edge deleted (set to INF) and
    an absent edge inserted, mixed with every other kind."""
    random_sequence(5000 + int(100 * density) + undirected, 170, undirected, 24, 200, density,
                    inf_edges=True)


@pytest.mark.parametrize("undirected", [False, True])
@pytest.mark.parametrize("limit", [1, 3])
def test_random_sequences_tiny_index(limit, undirected):
    """A 1- or 3-entry light-edge index forces the exhaustive in-edge scans."""
    random_sequence(2000 + limit + undirected, 160, undirected, 12, 50, 0.8, limit=limit)


@pytest.mark.parametrize("undirected", [False, True])
def test_largest_capacity(undirected):
    """A graph at the largest capacity (pitch APSP_MAX_CAPACITY): every update
    kind against the oracle, with weights 1..3 so that removals and tight
    increases flag many pairs and rows go to the heavy-row pass, whose LDS
    row then spans the whole pitch (close to the 160 KiB limit)."""
    from paper_2412_15122_amd import _native as N
    from paper_2412_15122_amd.apsp import Graph
    rng = np.random.default_rng(7100 + undirected)
    n = 260
    adj = W.random_graph(n, 1, 3, undirected=undirected, density=1.0, seed=int(rng.integers(1 << 30)))
    g = Graph(adj, undirected=undirected, capacity=N.APSP_MAX_CAPACITY)
    st = W.GraphState(adj, undirected)
    A, ids = adj.copy(), list(range(n))
    expect_equal(g, A, ids, "cold")
    heavy = 0
    kinds = [W.REMOVE, W.ADD, W.INCREASE, W.DECREASE] * 3
    for step, kind in enumerate(kinds):
        if kind == W.INCREASE:
            # the lightest edge on the most shortest paths: a tight increase
            u, v = 0, 1
            best = -1
            Dm = O.fw(A)
            for _ in range(40):
                a, b = (int(x) for x in rng.choice(len(ids), size=2, replace=False))
                if A[a, b] >= INF:
                    continue
                c = int(((Dm[:, a:a + 1] + A[a, b] + Dm[b:b + 1, :]) == Dm).sum())
                if c > best:
                    best, u, v = c, a, b
            upd = W.Update(W.INCREASE, u=ids[u], v=ids[v], w=int(A[u, v]) + 3, old=int(A[u, v]))
            st.set_weight(ids[u], ids[v], upd.w)
        else:
            upd = W.make_update(rng, st, kind, wmin=1, wmax=3, inc_max=6, density=1.0)
        A, ids = apply(g, A, ids, upd, undirected)
        heavy += g.stats()["heavy_rows"]
        expect_equal(g, A, ids, f"step {step} {upd.kind}")
    assert heavy > 0, "no update reached the heavy-row pass"
    g.close()


@pytest.mark.parametrize("undirected", [False, True])
def test_random_sequences_zero_weights_sparse(undirected):
    random_sequence(3000 + undirected, 120, undirected, 14, 4, density=0.08, zero=0.3)


def test_ragged_capacity_boundaries():
    """Capacities that are not multiples of the 128-wide tile, filled to the brim."""
    for n, cap in ((126, 130), (255, 257)):
        random_sequence(4000 + n, n, False, 8, 100, cap_extra=cap - n)


# ---------------------------------------------------------------------------
# masks and statistics
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("undirected", [False, True])
def test_remove_mask_statistics(undirected):
    rng = np.random.default_rng(77 + undirected)
    adj = W.random_graph(180, 1, 30, undirected=undirected, seed=9 + undirected)
    g = lib_graph(adj, undirected, capacity=200)
    A, ids = adj.copy(), list(range(180))
    for _ in range(4):
        D = O.fw(A)
        k = ids[int(rng.integers(len(ids)))]
        F = O.remove_mask(D, ids.index(k))
        phi, cost = O.remove_cost(F, len(ids))
        g.remove_node(k)
        s = g.stats()
        assert s["flagged"] == F.sum() and s["rows"] == phi and s["n_before"] == len(ids)
        assert abs(s["cost"] - cost) < 1e-12 and s["kind"] == 2
        A, ids = O.apply_update(A, ids, "remove", u=k, undirected=undirected)
    expect_equal(g, A, ids, "after removals")


@pytest.mark.parametrize("undirected", [False, True])
def test_refined_set_statistics(undirected):
    """|F'| and Phi' (the refined need_update list: pairs whose distance
    changed) after removals and tight edge increases, against the oracle's
    matrices before and after; small weights give many ties, so F' is much
    smaller than F, and rows with more than 32 flags take the heavy-row
    pass."""
    rng = np.random.default_rng(91 + undirected)
    n = 260
    adj = W.random_graph(n, 1, 12, undirected=undirected, seed=33 + undirected)
    g = lib_graph(adj, undirected, capacity=n)
    A, ids = adj.copy(), list(range(n))
    saw_heavy = False
    for step in range(8):
        D = O.fw(A)
        if step % 2 == 0:
            k = ids[int(rng.integers(len(ids)))]
            kc = ids.index(k)
            g.remove_node(k)
            A2, ids2 = O.apply_update(A, ids, "remove", u=k, undirected=undirected)
            keep = [t for t in range(len(ids)) if t != kc]
            R = O.refined_set(D[np.ix_(keep, keep)], O.fw(A2))
        else:
            tight = [(u, v) for u in range(len(ids)) for v in range(len(ids))
                     if u != v and A[u, v] == D[u, v] and A[u, v] < INF]
            u, v = tight[int(rng.integers(len(tight)))]
            w_new = int(A[u, v]) + 7
            g.update_edge(ids[u], ids[v], w_new)
            A2, ids2 = O.apply_update(A, ids, "edge", u=ids[u], v=ids[v], w=w_new, undirected=undirected)
            R = O.refined_set(D, O.fw(A2))
        s = g.stats()
        saw_heavy |= s["heavy_rows"] > 0
        phi = int(np.count_nonzero(R.any(axis=1)))
        assert s["changed"] == int(R.sum()) and s["rows_changed"] == phi, (step, s, int(R.sum()), phi)
        assert abs(s["cost_refined"] - phi / (len(ids) - 1)) < 1e-12
        assert s["changed"] <= s["flagged"] and s["rows_changed"] <= s["rows"]
        A, ids = A2, ids2
        expect_equal(g, A, ids, f"step {step}")
    assert saw_heavy


@pytest.mark.parametrize("undirected", [False, True])
def test_increase_statistics_read_after_copies(undirected):
    """A tight increase leaves its recompute statistics as per-work-group
    partials that are summed when first read: a clone and a grown copy made
    before that read, and the graph read after them, all report the refined
    set the oracle's matrices give; a removal that follows reports its own
    figures only."""
    n = 200
    rng = np.random.default_rng(61 + undirected)
    adj = W.random_graph(n, 1, 12, undirected=undirected, seed=61 + undirected)
    g = lib_graph(adj, undirected, capacity=n)
    A, ids = adj.copy(), list(range(n))
    D = O.fw(A)
    tight = [(u, v) for u in range(n) for v in range(n) if u != v and A[u, v] == D[u, v] and A[u, v] < INF]
    for _ in range(40):
        u, v = tight[int(rng.integers(len(tight)))]
        A2, ids2 = O.apply_update(A, ids, "edge", u=u, v=v, w=int(A[u, v]) + 7, undirected=undirected)
        R = O.refined_set(D, O.fw(A2))
        if R.sum() > 0:
            break
    assert R.sum() > 0
    g.update_edge(u, v, int(A[u, v]) + 7)
    c = g.clone()
    h = g.grow(n + 16)
    phi = int(np.count_nonzero(R.any(axis=1)))
    for x in (c, h, g):
        s = x.stats()
        assert s["kind"] == 4 and s["changed"] == int(R.sum()) and s["rows_changed"] == phi, s
    A, ids = A2, ids2
    expect_equal(c, A, ids, "clone")
    expect_equal(h, A, ids, "grown copy")
    c.close()
    h.close()
    D = O.fw(A)
    k = ids[int(rng.integers(len(ids)))]
    F = O.remove_mask(D, ids.index(k))
    g.remove_node(k)
    A2, ids2 = O.apply_update(A, ids, "remove", u=k, undirected=undirected)
    keep = [t for t in range(len(ids)) if t != ids.index(k)]
    R = O.refined_set(D[np.ix_(keep, keep)], O.fw(A2))
    s = g.stats()
    assert s["kind"] == 2 and s["flagged"] == F.sum() and s["changed"] == int(R.sum()), s
    expect_equal(g, A2, ids2, "removal")


@pytest.mark.parametrize("undirected", [False, True])
def test_edge_increase_mask_statistics(undirected):
    adj = W.random_graph(150, 1, 8, undirected=undirected, seed=21 + undirected)
    g = lib_graph(adj, undirected, capacity=150)
    A, ids = adj.copy(), list(range(150))
    D = O.fw(A)
    tight = [(u, v) for u in range(150) for v in range(150) if u != v and A[u, v] == D[u, v]]
    slack = [(u, v) for u in range(150) for v in range(150) if u != v and A[u, v] > D[u, v]]
    for (u, v) in tight[:3] + slack[:2]:
        D = O.fw(A)
        w_old = int(A[u, v])
        Fe = O.edge_mask(D, u, v, w_old, undirected)
        g.update_edge(u, v, w_old + 5)
        s = g.stats()
        if A[u, v] == D[u, v]:
            assert s["kind"] == 4 and s["flagged"] == Fe.sum()
        else:
            assert s["noop"] == 1 and s["flagged"] == 0 and Fe.sum() == 0
        A, ids = O.apply_update(A, ids, "edge", u=u, v=v, w=w_old + 5, undirected=undirected)
        expect_equal(g, A, ids, "increase")


def test_edge_decrease_noop_and_rows():
    adj = W.random_graph(140, 1, 100, seed=31)
    g = lib_graph(adj, False)
    A, ids = adj.copy(), list(range(140))
    D = O.fw(A)
    u, v = 3, 77
    g.update_edge(u, v, int(D[u, v]))          # not below D[u][v]: D cannot change
    s = g.stats()
    assert s["noop"] == 1 and s["rows_relaxed"] == 0
    A, ids = O.apply_update(A, ids, "edge", u=u, v=v, w=int(D[u, v]), undirected=False)
    expect_equal(g, A, ids)
    g.update_edge(u, v, 0)
    s = g.stats()
    rows = int(np.count_nonzero(O.oplus(D[:, u], 0) < D[:, v]))
    assert s["kind"] == 3 and s["rows_relaxed"] == rows
    A, ids = O.apply_update(A, ids, "edge", u=u, v=v, w=0, undirected=False)
    expect_equal(g, A, ids)


@pytest.mark.parametrize("undirected", [True, False])
def test_edge_scope_matches_oracle(undirected):
    adj = W.random_graph(130, 1, 6, undirected=undirected, seed=41)
    g = lib_graph(adj, undirected)
    D = O.fw(adj)
    if not undirected:
        assert not np.array_equal(D, D.T)
    for (u, v) in ((0, 1), (1, 0), (5, 99), (99, 5), (64, 65), (127, 128)):
        w = int(adj[u, v])
        assert g.edge_scope(u, v) == O.edge_scope(D[:, u], D[:, v], D[u, :], D[v, :], w), (u, v)


# ---------------------------------------------------------------------------
# Algorithm 5's switch, round trips, Algorithm 6's route
# ---------------------------------------------------------------------------

def test_fallback_policies_give_identical_matrices():
    from paper_2412_15122_amd import _native as N
    wl = W.config1()
    results = []
    for policy, delta in ((N.APSP_FALLBACK_NEVER, 0.5), (N.APSP_FALLBACK_COST, 0.0),
                          (N.APSP_FALLBACK_COST, 0.25), (N.APSP_FALLBACK_COST, 1.0),
                          (N.APSP_FALLBACK_ALWAYS, 0.5)):
        g = lib_graph(wl.adj, False, capacity=300)
        g.set_fallback(policy, delta)
        A, ids = wl.adj.copy(), list(range(256))
        for upd in wl.updates:
            A, ids = apply(g, A, ids, upd, False)
            if upd.kind == W.REMOVE:
                s = g.stats()
                if policy == N.APSP_FALLBACK_ALWAYS:
                    assert s["fallback"] == 1
                elif policy == N.APSP_FALLBACK_COST:
                    assert s["fallback"] == (s["cost"] > delta)
        results.append(g.matrix())
        expect_equal(g, A, ids, f"policy {policy} {delta}")
    for r in results[1:]:
        assert np.array_equal(r, results[0])


@pytest.mark.parametrize("undirected", [False, True])
def test_round_trips(undirected):
    rng = np.random.default_rng(5 + undirected)
    adj = W.random_graph(200, 1, 500, undirected=undirected, seed=51 + undirected)
    g = lib_graph(adj, undirected, capacity=210)
    D0 = g.matrix()
    # add p, then remove p: back to the original matrix
    w = rng.integers(1, 500, size=200).astype(np.int32)
    w_in = w if undirected else rng.integers(1, 500, size=200).astype(np.int32)
    p = g.add_node(w, w_in)
    g.remove_node(p)
    assert np.array_equal(g.matrix(), D0)
    # remove k, add it back with its old edges (new id): same matrix
    A = g.adjacency()
    k = 17
    keep = [x for x in range(200) if x != k]
    g.remove_node(k)
    nid = g.add_node(A[k, keep], A[keep, k])
    D1 = g.matrix()
    order = keep + [k]
    assert np.array_equal(D1, D0[np.ix_(order, order)]) and g.ids()[-1] == nid
    # decrease then increase back, and the reverse
    for (u, v) in ((1, 2), (30, 40)):
        before = g.matrix()
        old = int(g.adjacency()[g.ids().index(u), g.ids().index(v)])
        g.update_edge(u, v, 1)
        g.update_edge(u, v, old)
        assert np.array_equal(g.matrix(), before)
        g.update_edge(u, v, old + 300)
        g.update_edge(u, v, old)
        assert np.array_equal(g.matrix(), before)


@pytest.mark.parametrize("undirected", [False, True])
def test_update_edge_equals_algorithm6_route(undirected):
    """Algorithm 6 removes the endpoint that is cheaper to remove and adds it
    back with the new edge; composed from the library's own calls it must
    reach the same matrix as the direct update."""
    rng = np.random.default_rng(61 + undirected)
    adj = W.random_graph(150, 1, 30, undirected=undirected, seed=71 + undirected)
    for trial in range(3):
        u, v = (int(x) for x in rng.choice(150, size=2, replace=False))
        w_new = int(rng.integers(1, 60))
        direct = lib_graph(adj, undirected, capacity=152)
        direct.update_edge(u, v, w_new)
        Dd = direct.matrix()
        D = O.fw(adj)
        cost_u = O.remove_cost(O.remove_mask(D, u), 150)[1]
        cost_v = O.remove_cost(O.remove_mask(D, v), 150)[1]
        k = u if cost_u < cost_v else v          # a tie removes the second endpoint
        route = lib_graph(adj, undirected, capacity=152)
        A2 = adj.copy()
        A2[u, v] = w_new
        if undirected:
            A2[v, u] = w_new
        keep = [x for x in range(150) if x != k]
        route.remove_node(k)
        route.add_node(A2[k, keep], A2[keep, k])
        order = keep + [k]
        assert np.array_equal(route.matrix(), Dd[np.ix_(order, order)])


# ---------------------------------------------------------------------------
# query (Algorithm 7)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("undirected", [False, True])
def test_query_canonical_path(undirected):
    rng = np.random.default_rng(81 + undirected)
    for n, wmax, density in ((7, 3, 1.0), (90, 4, 0.4), (260, 1000, 1.0), (150, 2, 0.02)):
        adj = W.random_graph(n, 1, wmax, undirected=undirected, density=density, seed=int(rng.integers(1 << 30)))
        g = lib_graph(adj, undirected)
        D = O.fw(adj)
        for _ in range(25):
            i, j = (int(x) for x in rng.integers(0, n, size=2))
            dist, path = g.query(i, j)
            assert dist == D[i, j]
            assert path == O.canonical_path(adj, D, i, j)


def test_query_with_zero_weights_is_a_shortest_simple_path():
    rng = np.random.default_rng(91)
    adj = W.random_graph(120, 1, 3, density=0.3, zero_frac=0.5, seed=92)
    g = lib_graph(adj, False)
    D = O.fw(adj)
    for _ in range(40):
        i, j = (int(x) for x in rng.integers(0, 120, size=2))
        dist, path = g.query(i, j)
        assert dist == D[i, j]
        if D[i, j] >= INF:
            assert path == []
            continue
        assert path[0] == i and path[-1] == j and len(set(path)) == len(path)
        assert sum(int(adj[a, b]) for a, b in zip(path[:-1], path[1:])) == dist


# ---------------------------------------------------------------------------
# errors leave the graph unchanged
# ---------------------------------------------------------------------------

def test_errors_leave_graph_unchanged():
    from paper_2412_15122_amd import _native as N
    adj = W.random_graph(50, 1, 9, seed=101)
    g = lib_graph(adj, False, capacity=51)
    D0 = g.matrix()

    def status(fn, *a):
        try:
            fn(*a)
        except N.ApspError as e:
            return e.status
        return N.APSP_OK

    assert status(g.remove_node, 999) == N.APSP_E_NOT_FOUND
    assert status(g.update_edge, 1, 1, 5) == N.APSP_E_INVALID
    assert status(g.update_edge, 1, 2, -1) == N.APSP_E_INVALID
    assert status(g.update_edge, 1, 2, INF + 1) == N.APSP_E_INVALID
    assert status(g.update_edge, 1, 999, 3) == N.APSP_E_NOT_FOUND
    assert status(g.query, 1, 999) == N.APSP_E_NOT_FOUND
    assert status(g.set_index_limit, 0) == N.APSP_E_INVALID
    assert status(g.set_fallback, 9, 0.5) == N.APSP_E_INVALID
    assert np.array_equal(g.matrix(), D0) and g.ids() == list(range(50))
    p = g.add_node(np.full(50, 3, np.int32), np.full(50, 4, np.int32))
    assert p == 50
    assert status(g.add_node, np.full(51, 3, np.int32), np.full(51, 4, np.int32)) == N.APSP_E_CAPACITY
    g.remove_node(p)
    assert np.array_equal(g.matrix(), D0)
    g.remove_node(7)
    assert status(g.remove_node, 7) == N.APSP_E_NOT_FOUND
    g.sync()


def test_device_weight_out_of_range_is_reported():
    from paper_2412_15122_amd import _native as N
    adj = W.random_graph(30, 1, 9, seed=111)
    g = lib_graph(adj, False, capacity=31)
    w = np.full(30, 5, np.int32)
    w[4] = -3                                     # invalid: becomes an absent edge
    nid = g.add_node(w, np.full(30, 6, np.int32))
    with pytest.raises(N.ApspError) as e:
        g.sync()
    assert e.value.status == N.APSP_E_VALUE
    g.sync()                                      # reported once
    A, ids = O.apply_update(adj, list(range(30)), "add", w_out=np.where(w < 0, INF, w),
                            w_in=np.full(30, 6, np.int32))
    assert nid == 30
    expect_equal(g, A, ids)


def test_empty_graph_grows():
    g = lib_graph(np.zeros((0, 0), np.int32), False, capacity=4)
    assert g.num_nodes() == 0
    a = g.add_node([], [])
    b = g.add_node([7], [9])
    c = g.add_node([1, INF], [2, 3])
    A = np.array([[0, 9, 2], [7, 0, 3], [1, INF, 0]], dtype=np.int32)
    expect_equal(g, A, [a, b, c])
    g.remove_node(b)
    A2, ids2 = O.apply_update(A, [0, 1, 2], "remove", u=1)
    expect_equal(g, A2, ids2)
    g.remove_node(a)
    g.remove_node(c)
    assert g.num_nodes() == 0
    assert g.add_node([], []) == 3


def test_reads_on_another_stream_see_queued_updates():
    """A graph whose work runs on a side stream: additions (host weight
    vectors) and removals queued there, then the matrices read from the
    default stream with no synchronization by the caller."""
    import torch
    rng = np.random.default_rng(77)
    n = 300
    adj = W.random_graph(n, 1, 1000, seed=77)
    g = lib_graph(adj, False, capacity=n + 40)
    side = torch.cuda.Stream()
    g.set_stream(side)
    st = W.GraphState(adj, False)
    A, ids = adj.copy(), list(range(n))
    for step in range(24):
        kind = (W.ADD, W.REMOVE, W.INCREASE, W.DECREASE)[step % 4]
        upd = W.make_update(rng, st, kind, wmin=1, wmax=1000, inc_max=2000)
        A, ids = apply(g, A, ids, upd, False)
    expect_equal(g, A, ids, "after queued updates on a side stream")
    g.sync()
