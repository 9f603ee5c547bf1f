"""Pins of the CPU oracle to things other than itself.

Each test checks the oracle against what the paper or the mathematics fixes:
brute-force enumeration of simple paths, an external library (scipy's
Floyd-Warshall), the Bellman optimality equations (unique solution for
positive weights), the paper's add-node theorems rebuilt in plain loops, and
the paper's printed worked example.  A plausible slip in the oracle (dropped
term, swapped index, wrong comparison) fails at least one of them.
"""
import json
import os

import numpy as np
import pytest

from oracle import oracle as O
from paper_2412_15122_amd import workloads as W

INF = O.INF
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def rand_graph(rng, n, wmax, *, undirected=False, density=1.0, zero=0.0):
    return W.random_graph(n, 1, wmax, undirected=undirected, density=density,
                          seed=int(rng.integers(1 << 31)), zero_frac=zero)


# ---------------------------------------------------------------------------
# cold APSP: three independent routes agree
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("n", [0, 1, 2, 3, 5, 7])
@pytest.mark.parametrize("undirected", [False, True])
def test_fw_equals_brute_force(n, undirected):
    rng = np.random.default_rng(100 + n + 10 * undirected)
    for trial in range(6):
        density = [1.0, 0.6, 0.3][trial % 3]
        wmax = [3, 20, 1000][trial % 3]            # [1,3] forces heavy ties
        zero = 0.2 if trial == 4 else 0.0           # zero-weight edges are allowed
        A = rand_graph(rng, n, wmax, undirected=undirected, density=density, zero=zero)
        assert np.array_equal(O.fw(A), O.brute_force_apsp(A))


@pytest.mark.parametrize("n", [2, 17, 64, 150])
def test_fw_equals_scipy(n):
    from scipy.sparse.csgraph import floyd_warshall
    rng = np.random.default_rng(7 + n)
    for density in (1.0, 0.4, 0.05):
        A = rand_graph(rng, n, 50, density=density)
        Af = np.where(A >= INF, np.inf, A.astype(np.float64))
        np.fill_diagonal(Af, 0.0)
        ref = floyd_warshall(Af, directed=True)
        ref = np.where(np.isinf(ref), INF, ref).astype(np.int64)
        assert np.array_equal(O.fw(A).astype(np.int64), ref)


@pytest.mark.parametrize("threads", [1, 3])
def test_dijkstra_rows_equal_fw(threads):
    rng = np.random.default_rng(3)
    for n, density in ((1, 1.0), (40, 0.3), (200, 1.0), (257, 0.9)):
        A = rand_graph(rng, n, 100, density=density)
        D = O.fw(A, threads=threads)
        srcs = np.arange(n)
        assert np.array_equal(O.dijkstra_rows(A, srcs, threads=threads), D)
        assert np.array_equal(O.dijkstra_cols(A, srcs, threads=threads), D.T)


def test_fw_pivot_ranges_compose():
    rng = np.random.default_rng(4)
    A = rand_graph(rng, 90, 30, density=0.5)
    D = O.fw_init(A)
    for k0 in range(0, 90, 17):
        O.fw_pivots(D, k0, min(90, k0 + 17), threads=2)
    assert np.array_equal(D, O.fw(A))


def test_fw_rejects_out_of_range_weights():
    A = np.zeros((3, 3), dtype=np.int32)
    A[0, 1] = -1
    with pytest.raises(ValueError):
        O.fw(A)
    A[0, 1] = INF + 1
    with pytest.raises(ValueError):
        O.fw(A)


def bfs_reachable(A):
    n = A.shape[0]
    R = np.zeros((n, n), dtype=bool)
    for s in range(n):
        seen = {s}
        stack = [s]
        while stack:
            x = stack.pop()
            for y in range(n):
                if A[x, y] < INF and y not in seen:
                    seen.add(y)
                    stack.append(y)
        R[s, list(seen)] = True
    return R


@pytest.mark.parametrize("undirected", [False, True])
def test_fw_invariants_bellman_unique(undirected):
    """With w >= 1 the Bellman equations D[i][i] = 0,
    D[i][j] = min_t A[i][t] (+) D[t][j] have exactly one solution (the APSP
    matrix), so checking them pins every entry.  Reachability comes from an
    independent graph search."""
    rng = np.random.default_rng(11)
    for n, density, wmax in ((60, 1.0, 10), (80, 0.1, 1000), (45, 0.03, 5)):
        A = rand_graph(rng, n, wmax, undirected=undirected, density=density)
        D = O.fw(A).astype(np.int64)
        A64 = A.astype(np.int64)
        assert np.all(np.diag(D) == 0)
        off = ~np.eye(n, dtype=bool)
        assert np.all(D[off] <= A64[off])
        # triangle inequality
        for k in range(n):
            assert np.all(D <= O.oplus(D[:, k][:, None], D[k, :][None, :]))
        # Bellman optimality (first hop)
        best = np.full((n, n), INF, dtype=np.int64)
        for t in range(n):
            best = np.minimum(best, O.oplus(A64[:, t][:, None], D[t, :][None, :]))
        assert np.array_equal(D[off], best[off])
        assert np.array_equal(D < INF, bfs_reachable(A))
        if undirected:
            assert np.array_equal(D, D.T)


# ---------------------------------------------------------------------------
# the paper's add-node theorems, written out, reproduce the oracle
# ---------------------------------------------------------------------------

def apsp_by_repeated_add(A):
    """Cold APSP by adding nodes one at a time (the recursion the paper's
    Algorithm 1 rests on): the new row by Theorem 1, the new column
    by Theorem 2, old pairs by Theorem 3.  Plain loops,
    no shared code with the oracle."""
    n = A.shape[0]
    M = [[0]]
    for m in range(1, n):
        out = []
        for r in range(m):      # SPD(new, r) = min_t d(new, t) + SPD(t, r)
            out.append(min(min(int(A[m, t]) + M[t][r] for t in range(m)), INF))
        inn = []
        for r in range(m):      # SPD(r, new) = min_t SPD(r, t) + d(t, new)
            inn.append(min(min(M[r][t] + int(A[t, m]) for t in range(m)), INF))
        for i in range(m):      # SPD'(i, j) = min(SPD(i, j), t1 + t2)
            for j in range(m):
                M[i][j] = min(M[i][j], inn[i] + out[j])
        for i in range(m):
            M[i].append(inn[i])
        M.append(out + [0])
    return np.array(M, dtype=np.int64).reshape(n, n) if n else np.zeros((0, 0), np.int64)


@pytest.mark.parametrize("n", [1, 2, 9, 33])
def test_repeated_add_node_equals_fw(n):
    rng = np.random.default_rng(21 + n)
    for density in (1.0, 0.3):
        A = rand_graph(rng, n, 40, density=density)
        assert np.array_equal(apsp_by_repeated_add(A), O.fw(A).astype(np.int64))


# ---------------------------------------------------------------------------
# the paper's worked example (printed need_update_lists)
# ---------------------------------------------------------------------------

def load_fixture():
    with open(os.path.join(GOLDEN, "paper_remove_example.json")) as f:
        fx = json.load(f)
    names = fx["nodes"]
    idx = {c: i for i, c in enumerate(names)}
    n = len(names)
    A = np.full((n, n), INF, dtype=np.int32)
    np.fill_diagonal(A, 0)
    for a, b, w in fx["undirected_edges"]:
        A[idx[a], idx[b]] = A[idx[b], idx[a]] = w
    return fx, names, idx, A


def test_paper_worked_example_need_update_lists():
    fx, names, idx, A = load_fixture()
    D = O.fw(A)
    for removed, exp in fx["remove"].items():
        k = idx[removed]
        F = O.remove_mask(D, k)
        got = {names[i]: [[names[i], names[j]] for j in range(len(names)) if F[i, j]]
               for i in range(len(names)) if i != k}
        assert got == exp["need_update_list"]
        A2, ids2 = O.apply_update(A, list(range(4)), "remove", u=k, undirected=True)
        D2 = O.fw(A2)
        pos = {i: p for p, i in enumerate(ids2)}
        for a, b in exp["equal"]:
            assert D[idx[a], idx[b]] == D2[pos[idx[a]], pos[idx[b]]]
        for a, b in exp["not_equal"]:
            assert D[idx[a], idx[b]] != D2[pos[idx[a]], pos[idx[b]]]


def test_paper_worked_example_cost():
    fx, names, idx, A = load_fixture()
    D = O.fw(A)
    assert O.remove_cost(O.remove_mask(D, idx["C"]), 4) == (0, 0.0)
    assert O.remove_cost(O.remove_mask(D, idx["B"]), 4) == (3, 1.0)


# ---------------------------------------------------------------------------
# masks: exact contents by brute force, soundness by cold recompute
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("undirected", [False, True])
def test_remove_mask_is_node_on_some_shortest_path(undirected):
    """For w >= 1, D[i][k] + D[k][j] == D[i][j] exactly when k lies on some
    shortest simple i->j path (enumerated)."""
    rng = np.random.default_rng(31)
    for trial in range(8):
        n = 6
        A = rand_graph(rng, n, [2, 9][trial % 2], undirected=undirected,
                       density=[1.0, 0.5][trial % 2 == 1 and trial > 3])
        D = O.fw(A)
        for k in range(n):
            F = O.remove_mask(D, k)
            for i in range(n):
                for j in range(n):
                    on = (i != j and k not in (i, j) and
                          any(k in p for p in O.all_shortest_simple_paths(A, i, j)))
                    assert F[i, j] == on, (trial, k, i, j)


@pytest.mark.parametrize("undirected", [False, True])
def test_edge_mask_is_edge_on_some_shortest_path(undirected):
    rng = np.random.default_rng(41)
    for trial in range(8):
        n = 6
        A = rand_graph(rng, n, [2, 9][trial % 2], undirected=undirected)
        D = O.fw(A)
        for u in range(n):
            for v in range(n):
                if u == v:
                    continue
                F = O.edge_mask(D, u, v, int(A[u, v]), undirected)
                for i in range(n):
                    for j in range(n):
                        on = False
                        if i != j:
                            for p in O.all_shortest_simple_paths(A, i, j):
                                hops = list(zip(p[:-1], p[1:]))
                                if (u, v) in hops or (undirected and (v, u) in hops):
                                    on = True
                        assert F[i, j] == on, (trial, u, v, i, j)


@pytest.mark.parametrize("undirected", [False, True])
def test_masks_cover_every_changed_pair(undirected):
    """Corollary 3 (soundness): pairs outside the mask keep their
    distance.  Checked against a cold recompute, with ties and zero weights."""
    rng = np.random.default_rng(51)
    for trial in range(12):
        n = int(rng.integers(2, 40))
        A = rand_graph(rng, n, [3, 50][trial % 2], undirected=undirected,
                       density=[1.0, 0.4][trial % 3 == 0], zero=0.1 if trial % 4 == 1 else 0.0)
        D = O.fw(A)
        ids = list(range(n))
        k = int(rng.integers(n))
        F = O.remove_mask(D, k)
        A2, ids2 = O.apply_update(A, ids, "remove", u=k, undirected=undirected)
        D2 = O.fw(A2)
        keep = [x for x in range(n) if x != k]
        changed = D[np.ix_(keep, keep)] != D2
        assert not np.any(changed & ~F[np.ix_(keep, keep)])
        u, v = rng.choice(n, size=2, replace=False)
        if A[u, v] < INF:
            w_new = int(A[u, v]) + int(rng.integers(1, 100))
            Fe = O.edge_mask(D, u, v, int(A[u, v]), undirected)
            A3, _ = O.apply_update(A, ids, "increase", u=u, v=v, w=w_new, undirected=undirected)
            assert not np.any((O.fw(A3) != D) & ~Fe)


# ---------------------------------------------------------------------------
# query
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("undirected", [False, True])
def test_canonical_path_is_lexicographic_minimum(undirected):
    rng = np.random.default_rng(61)
    for trial in range(10):
        n = int(rng.integers(1, 8))
        A = rand_graph(rng, n, [2, 30][trial % 2], undirected=undirected,
                       density=[1.0, 0.5][trial % 3 == 0])
        D = O.fw(A)
        for i in range(n):
            for j in range(n):
                paths = O.all_shortest_simple_paths(A, i, j)
                got = O.canonical_path(A, D, i, j)
                if not paths:
                    assert got == [] and D[i, j] == INF
                else:
                    assert tuple(got) == paths[0]


def test_edge_scope_counts():
    rng = np.random.default_rng(71)
    A = rand_graph(rng, 30, 5, undirected=True)
    D = O.fw(A)
    for (u, v) in ((0, 1), (3, 7), (10, 2)):
        w = int(A[u, v])
        R, C = O.edge_scope(D[:, u], D[:, v], D[u, :], D[v, :], w)
        assert R == sum(1 for i in range(30) if min(D[i, u] + w, INF) == D[i, v] < INF)
        assert C == sum(1 for j in range(30) if min(w + D[v, j], INF) == D[u, j] < INF)
        # |F_e| never exceeds |R| * |C| in either direction
        Fe = O.edge_mask(D, u, v, w, False)
        assert Fe.sum() <= R * C


@pytest.mark.parametrize("undirected", [False, True])
def test_edge_scope_by_brute_force(undirected):
    """|R| and |C| against their meaning, by enumerating every shortest simple
    path on small graphs: R = the sources i with some shortest i->v path whose
    last edge is u->v, C = the targets j with some shortest u->j path whose
    first edge is u->v.  On a directed graph D is not symmetric, so a row read
    where a column belongs (or the reverse) changes the counts."""
    rng = np.random.default_rng(72 + undirected)
    checked = 0
    for trial in range(14):
        n = 5 + trial % 3
        A = rand_graph(rng, n, [2, 4, 9][trial % 3], undirected=undirected, density=0.75)
        D = O.fw(A)
        for u in range(n):
            for v in range(n):
                if u == v or A[u, v] >= INF:
                    continue
                w = int(A[u, v])
                R = sum(1 for i in range(n)
                        if any(p[-2:] == (u, v) for p in O.all_shortest_simple_paths(A, i, v)))
                C = sum(1 for j in range(n)
                        if any(p[:2] == (u, v) for p in O.all_shortest_simple_paths(A, u, j)))
                assert O.edge_scope(D[:, u], D[:, v], D[u, :], D[v, :], w) == (R, C), (trial, u, v)
                checked += 1
    assert checked > 100


# ---------------------------------------------------------------------------
# the updated graph G'
# ---------------------------------------------------------------------------

def test_apply_update_semantics():
    A = np.array([[0, 5, INF], [2, 0, 7], [1, INF, 0]], dtype=np.int32)
    ids = [0, 4, 9]
    B, ids2 = O.apply_update(A, ids, "add", w_out=[3, 4, 5], w_in=[6, 7, 8])
    assert ids2 == [0, 4, 9, 10]
    assert B[3, :3].tolist() == [3, 4, 5] and B[:3, 3].tolist() == [6, 7, 8] and B[3, 3] == 0
    C, ids3 = O.apply_update(B, ids2, "remove", u=4)
    assert ids3 == [0, 9, 10]
    assert C.tolist() == [[0, INF, 6], [1, 0, 8], [3, 5, 0]]
    E, _ = O.apply_update(C, ids3, "decrease", u=9, v=0, w=0, undirected=True)
    assert E[1, 0] == 0 and E[0, 1] == 0
    assert O.apply_update(np.zeros((0, 0), np.int32), [], "add", w_out=[], w_in=[])[1] == [0]


# ---------------------------------------------------------------------------
# the refined need_update list (Algorithms 11-12, Theorem 6)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("undirected", [False, True])
def test_refined_set_is_pairs_whose_every_shortest_path_uses_k(undirected):
    """Brute force over simple paths (n <= 7, small weights: many ties): the
    pairs whose distance changes when k is removed are exactly those whose
    every shortest simple path passes through k, and they lie inside the
    need_update list."""
    rng = np.random.default_rng(123 + undirected)
    for trial in range(25):
        n = int(rng.integers(3, 8))
        A = W.random_graph(n, 1, 3, undirected=undirected, density=float(rng.uniform(0.4, 1.0)),
                           seed=int(rng.integers(1 << 30)))
        D = O.fw(A)
        k = int(rng.integers(n))
        keep = [t for t in range(n) if t != k]
        A2 = A[np.ix_(keep, keep)]
        R = O.refined_set(D[np.ix_(keep, keep)], O.fw(A2))
        F = O.remove_mask(D, k)[np.ix_(keep, keep)]
        assert not (R & ~F).any(), "a changed pair outside the need_update list"
        for a, i in enumerate(keep):
            for b, j in enumerate(keep):
                if i == j:
                    continue
                paths = O.all_shortest_simple_paths(A, i, j)
                all_use_k = bool(paths) and all(k in p[1:-1] for p in paths)
                assert R[a, b] == all_use_k, (trial, i, j, k)


@pytest.mark.parametrize("undirected", [False, True])
def test_refined_set_of_a_raised_edge_is_pairs_whose_every_shortest_path_uses_it(undirected):
    rng = np.random.default_rng(321 + undirected)
    for trial in range(25):
        n = int(rng.integers(3, 8))
        A = W.random_graph(n, 1, 3, undirected=undirected, density=1.0, seed=int(rng.integers(1 << 30)))
        D = O.fw(A)
        u, v = (int(x) for x in rng.choice(n, 2, replace=False))
        w_new = int(A[u, v]) + int(rng.integers(1, 4))
        A2, _ = O.apply_update(A, list(range(n)), "edge", u=u, v=v, w=w_new, undirected=undirected)
        R = O.refined_set(D, O.fw(A2))
        F = O.edge_mask(D, u, v, int(A[u, v]), undirected)
        assert not (R & ~F).any()

        def uses(p):
            steps = list(zip(p[:-1], p[1:]))
            return (u, v) in steps or (undirected and (v, u) in steps)

        for i in range(n):
            for j in range(n):
                if i == j:
                    continue
                paths = O.all_shortest_simple_paths(A, i, j)
                assert R[i, j] == (bool(paths) and all(uses(p) for p in paths)), (trial, i, j, u, v)


# ---------------------------------------------------------------------------
# nodes of the shortest paths of a pair (Algorithms 7, 8, 10)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("undirected", [False, True])
@pytest.mark.parametrize("zero", [0.0, 0.3])
def test_pair_nodes_against_all_shortest_simple_paths(undirected, zero):
    """Brute force over simple paths (n <= 7, small weights: many ties; with
    and without zero-weight edges): key nodes are the intersection of all
    shortest simple paths without the endpoints; with positive weights the
    candidate set is their union, with zero weights it contains it."""
    rng = np.random.default_rng(7 + undirected + int(10 * zero))
    for trial in range(40):
        n = int(rng.integers(2, 8))
        A = W.random_graph(n, 1, 3, undirected=undirected, density=float(rng.uniform(0.3, 1.0)),
                           seed=int(rng.integers(1 << 30)), zero_frac=zero)
        D = O.fw(A)
        i, j = (int(x) for x in rng.integers(0, n, size=2))
        on, key = O.pair_nodes(A, D, i, j)
        if i == j:
            assert on == [i] and key == []
            continue
        paths = O.all_shortest_simple_paths(A, i, j)
        if not paths:
            assert on == [] and key == [] and D[i, j] >= INF
            continue
        union = sorted(set().union(*map(set, paths)))
        inter = sorted(set.intersection(*map(set, paths)) - {i, j})
        assert key == inter, (trial, i, j)
        if zero == 0.0:
            assert on == union, (trial, i, j)
        else:
            assert set(union) <= set(on)


def test_pair_nodes_of_a_path_graph():
    """A chain with a shortcut: 0-1-2-3-4, plus 1->3 of the same length as
    1-2-3: every node is on a shortest 0->4 path, 1 and 3 are key nodes, 2
    is not."""
    A = np.full((5, 5), INF, dtype=np.int32)
    for a, b in ((0, 1), (1, 2), (2, 3), (3, 4)):
        A[a, b] = 1
    A[1, 3] = 2
    D = O.fw(A)
    on, key = O.pair_nodes(A, D, 0, 4)
    assert on == [0, 1, 2, 3, 4] and key == [1, 3]


@pytest.mark.parametrize("zero", [0.0, 0.3])
def test_key_nodes_decide_removals(zero):
    """What Algorithm 10 uses the key nodes for: removing a key node of (i, j)
    raises D[i][j]; removing any other node leaves it (checked by a cold
    Floyd-Warshall of the graph without that node)."""
    rng = np.random.default_rng(41 + int(10 * zero))
    for trial in range(25):
        n = int(rng.integers(3, 12))
        A = W.random_graph(n, 1, 3, density=float(rng.uniform(0.2, 0.7)), seed=int(rng.integers(1 << 30)),
                           zero_frac=zero)
        D = O.fw(A)
        i, j = (int(x) for x in rng.choice(n, size=2, replace=False))
        on, key = O.pair_nodes(A, D, i, j)
        for k in range(n):
            if k in (i, j):
                continue
            keep = [t for t in range(n) if t != k]
            D2 = O.fw(A[np.ix_(keep, keep)])
            d2 = D2[keep.index(i), keep.index(j)]
            if k in key:
                assert d2 > D[i, j], (trial, k)
            else:
                assert d2 == D[i, j], (trial, k)


# ---------------------------------------------------------------------------
# minimax (bottleneck) paths: the (min, max) variant
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("undirected", [False, True])
def test_minimax_three_ways(undirected):
    """Floyd-Warshall with max = brute force over simple paths (n <= 7) =
    least reachability threshold (n <= 40); zero weights and many ties."""
    rng = np.random.default_rng(61 + undirected)
    for trial in range(30):
        n = int(rng.integers(1, 8)) if trial < 20 else int(rng.integers(8, 40))
        A = W.random_graph(n, 1, int(rng.integers(1, 20)), undirected=undirected,
                           density=float(rng.uniform(0.1, 0.9)), seed=int(rng.integers(1 << 30)),
                           zero_frac=0.15 if trial % 3 == 0 else 0.0)
        D = O.minimax_apsp(A)
        assert np.array_equal(D, O.minimax_by_thresholds(A)), trial
        if n <= 7:
            assert np.array_equal(D, O.brute_force_minimax(A)), trial


def test_minimax_undirected_equals_spanning_tree_bottleneck():
    """Undirected, positive weights: MM(i,j) is the largest edge on the
    path between i and j in a minimum spanning forest (scipy's)."""
    from scipy.sparse.csgraph import minimum_spanning_tree
    rng = np.random.default_rng(71)
    for trial in range(8):
        n = int(rng.integers(5, 60))
        A = W.random_graph(n, 1, 1000, undirected=True, density=float(rng.uniform(0.05, 0.6)),
                           seed=int(rng.integers(1 << 30)))
        dense = np.where(A >= INF, 0, A).astype(np.float64)
        np.fill_diagonal(dense, 0)
        T = minimum_spanning_tree(dense).toarray()
        T = np.maximum(T, T.T)
        want = np.full((n, n), INF, dtype=np.int64)
        for s in range(n):           # largest edge on the tree path from s
            want[s, s] = 0
            stack = [s]
            while stack:
                x = stack.pop()
                for y in np.nonzero(T[x])[0]:
                    if want[s, y] == INF:
                        want[s, y] = max(want[s, x], int(T[x, y]))
                        stack.append(int(y))
        assert np.array_equal(O.minimax_apsp(A), want), trial


def test_minimax_removal_mask_holds_every_change():
    """Corollary 3 with max: pairs outside the minimax mask of k keep
    their distance when k is removed."""
    rng = np.random.default_rng(81)
    for trial in range(20):
        n = int(rng.integers(3, 30))
        A = W.random_graph(n, 1, 6, density=float(rng.uniform(0.1, 0.8)), seed=int(rng.integers(1 << 30)))
        D = O.minimax_apsp(A)
        k = int(rng.integers(n))
        keep = [x for x in range(n) if x != k]
        D2 = O.minimax_apsp(A[np.ix_(keep, keep)])
        F = O.remove_mask(D, k, minimax=True)[np.ix_(keep, keep)]
        assert np.array_equal(D2[~F], D[np.ix_(keep, keep)][~F]), trial


def test_minimax_edge_mask_holds_every_change():
    """Corollary 3 with max, applied to the relay node of an edge: when an
    edge is raised, pairs outside its minimax mask keep their distance; and
    raising an edge heavier than its endpoints' minimax distance changes no
    distance at all (the rule that skips such an increase)."""
    rng = np.random.default_rng(83)
    for trial in range(20):
        n = int(rng.integers(3, 30))
        und = bool(trial % 2)
        A = W.random_graph(n, 1, 6, undirected=und, density=float(rng.uniform(0.2, 0.9)),
                           seed=int(rng.integers(1 << 30)))
        D = O.minimax_apsp(A)
        edges = np.argwhere((A < INF) & ~np.eye(n, dtype=bool))
        if len(edges) == 0:
            continue
        u, v = (int(x) for x in edges[int(rng.integers(len(edges)))])
        F = O.edge_mask(D, u, v, int(A[u, v]), und, minimax=True)
        A2 = A.copy()
        A2[u, v] = int(A[u, v]) + int(rng.integers(1, 8))
        if und:
            A2[v, u] = A2[u, v]
        D2 = O.minimax_apsp(A2)
        assert np.array_equal(D2[~F], D[~F]), trial
        if A[u, v] > D[u, v]:
            assert np.array_equal(D2, D), trial


def test_minimax_rows_equal_floyd_warshall():
    rng = np.random.default_rng(91)
    for trial in range(12):
        n = int(rng.integers(1, 70))
        A = W.random_graph(n, 1, int(rng.integers(1, 30)), undirected=bool(trial % 2),
                           density=float(rng.uniform(0.05, 0.9)), seed=int(rng.integers(1 << 30)),
                           zero_frac=0.1 if trial % 3 == 0 else 0.0)
        D = O.minimax_apsp(A)
        srcs = [int(x) for x in rng.integers(0, n, size=min(n, 5))]
        assert np.array_equal(O.minimax_rows(A, srcs), D[srcs]), trial


@pytest.mark.parametrize("undirected", [False, True])
def test_minimax_pair_nodes_against_brute_force(undirected):
    """Minimax pairs (n <= 7, small weights, zero weights too): the key nodes
    are the intersection of all simple paths whose largest edge is the
    minimax distance, those paths lie inside the node set, and removing a
    node raises the distance exactly when it is a key node."""
    rng = np.random.default_rng(101 + undirected)
    for trial in range(60):
        n = int(rng.integers(2, 8))
        A = W.random_graph(n, 1, 4, undirected=undirected, density=float(rng.uniform(0.3, 1.0)),
                           seed=int(rng.integers(1 << 30)), zero_frac=0.2 if trial % 2 else 0.0)
        D = O.minimax_apsp(A)
        i, j = (int(x) for x in rng.integers(0, n, size=2))
        on, key = O.minimax_pair_nodes(A, D, i, j)
        if i == j:
            assert on == [i] and key == []
            continue
        if D[i, j] >= INF:
            assert on == [] and key == []
            continue
        paths = [p for p, L in O._simple_paths(A, i, j)
                 if L < INF and max((int(A[a, b]) for a, b in zip(p, p[1:])), default=0) == D[i, j]]
        assert paths
        assert key == sorted(set.intersection(*map(set, paths)) - {i, j}), trial
        assert set().union(*map(set, paths)) <= set(on)
        assert key == [t for t in on if t not in (i, j) and O.minimax_key_test(A, i, j, int(D[i, j]), t)]
        for k in range(n):
            if k in (i, j):
                continue
            keep = [t for t in range(n) if t != k]
            d2 = O.minimax_apsp(A[np.ix_(keep, keep)])[keep.index(i), keep.index(j)]
            assert (d2 > D[i, j]) == (k in key), (trial, k)


@pytest.mark.parametrize("minimax", [False, True])
@pytest.mark.parametrize("undirected", [False, True])
def test_true_distance_matrices_pass_the_import_checks(undirected, minimax):
    """The O(n^2) conditions apsp_import checks hold for every true distance
    matrix (so a correct matrix is never refused): entries in [0, INF], a zero
    diagonal, no entry above its edge, symmetry when undirected -- here on
    graphs with absent edges, zero weights and unreachable pairs."""
    INF = W.INF
    rng = np.random.default_rng(5 + 2 * undirected + minimax)
    for n, density, zero in ((1, 1.0, 0.0), (9, 0.3, 0.3), (40, 0.1, 0.2), (60, 1.0, 0.0)):
        adj = W.random_graph(n, 1, 50, undirected=undirected, density=density,
                             seed=int(rng.integers(1 << 30)), zero_frac=zero)
        D = O.minimax_apsp(adj) if minimax else O.fw(adj)
        A = adj.astype(np.int64).copy()
        np.fill_diagonal(A, 0)
        assert D.min() >= 0 and D.max() <= INF
        assert np.all(np.diag(D) == 0)
        assert np.all(D.astype(np.int64) <= A)
        if undirected:
            assert np.array_equal(D, D.T)


# ---------------------------------------------------------------------------
# widest (maximum-capacity) paths
# ---------------------------------------------------------------------------

def rand_caps(rng, n, cmax, *, undirected=False, density=1.0, zero=0.0):
    """Capacities U[1, cmax] (some 0 with `zero`), absent edges INF."""
    return W.random_graph(n, 1, cmax, undirected=undirected, density=density,
                          seed=int(rng.integers(1 << 31)), zero_frac=zero)


@pytest.mark.parametrize("undirected", [False, True])
def test_widest_equals_brute_force_and_thresholds(undirected):
    rng = np.random.default_rng(301 + undirected)
    for trial in range(18):
        n = [0, 1, 2, 4, 6, 7][trial % 6]
        C = rand_caps(rng, n, [3, 50, O.WIDEST_TOP][trial % 3], undirected=undirected,
                      density=[1.0, 0.5, 0.25][trial % 3], zero=0.2 if trial % 4 == 1 else 0.0)
        Wf = O.widest_apsp(C)
        assert np.array_equal(Wf, O.brute_force_widest(C)), trial
        assert np.array_equal(Wf, O.widest_by_thresholds(C)), trial


def test_widest_by_maximum_spanning_tree():
    """Undirected: the width of a pair is the smallest capacity on its path
    in a maximum spanning forest (scipy's minimum spanning tree of
    (WIDEST_TOP + 1) - c, so every present edge stays positive)."""
    from scipy.sparse import csr_matrix
    from scipy.sparse.csgraph import minimum_spanning_tree, breadth_first_order
    rng = np.random.default_rng(305)
    for n, cmax, dens in ((40, 30, 1.0), (60, 1000, 0.15), (25, 4, 0.5)):
        C = rand_caps(rng, n, cmax, undirected=True, density=dens)
        M = np.where(C < INF, (O.WIDEST_TOP + 1) - C.astype(np.int64), 0).astype(np.float64)
        np.fill_diagonal(M, 0)
        T = minimum_spanning_tree(csr_matrix(M)).toarray()
        T = np.maximum(T, T.T)
        Wf = O.widest_apsp(C)
        for i in range(n):
            order, pred = breadth_first_order(csr_matrix(T), i, directed=False, return_predecessors=True)
            for j in range(n):
                if i == j:
                    assert Wf[i, j] == O.WIDEST_TOP
                elif j not in set(order.tolist()):
                    assert Wf[i, j] == INF
                else:
                    x, m = j, O.WIDEST_TOP
                    while x != i:
                        m = min(m, int(C[pred[x], x]))
                        x = pred[x]
                    assert Wf[i, j] == m, (i, j)


def test_widest_is_a_minimax_problem_on_flipped_capacities():
    """The reading the library takes: W = TOP - MM(TOP - C) entrywise
    (INF kept), checked here between two independent oracle routines."""
    rng = np.random.default_rng(309)
    for undirected in (False, True):
        C = rand_caps(rng, 30, 500, undirected=undirected, density=0.4, zero=0.1)
        F = np.where(C < INF, O.WIDEST_TOP - C.astype(np.int64), INF).astype(np.int32)
        MM = O.minimax_apsp(F).astype(np.int64)
        assert np.array_equal(O.widest_apsp(C), np.where(MM < INF, O.WIDEST_TOP - MM, INF))
