"""The paper's own warm-start procedures on the CPU (Algorithms 5, 6, 7, 11;
paper_cpu/procedures.c), pinned to the oracle: every result equals the oracle's
cold Floyd-Warshall of the updated graph, on both branches of the delta test;
Phi and Cost equal the need_update_list's by definition; Algorithm 11's list
lies inside Algorithm 5's and still holds every pair whose distance changes;
Algorithm 7's path is a shortest path."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_cpu import procedures as PC
from paper_2412_15122_amd import workloads as W

INF = W.INF


def graphs():
    rng = np.random.default_rng(5)
    for t in range(14):
        n = int(rng.integers(2, 90))
        und = bool(t % 2)
        wmax = (3, 10000)[t % 3 == 0]
        dens = (1.0, 0.3, 0.08)[t % 3]
        zero = 0.2 if t % 5 == 4 else 0.0
        A = W.random_graph(n, 1, wmax, undirected=und, density=dens, seed=int(rng.integers(1 << 30)),
                           zero_frac=zero)
        yield t, A, und, rng


@pytest.mark.parametrize("delta", [0.0, 0.5, 1.0])
def test_remove_and_remove_key_equal_cold(delta):
    for t, A, und, rng in graphs():
        n = A.shape[0]
        D = O.fw(A)
        assert np.array_equal(PC.fw(A)[0], D)
        k = int(rng.integers(n))
        A2, _ = O.apply_update(A, list(range(n)), "remove", u=k)
        want = O.fw(A2)
        F = O.remove_mask(D, k)
        phi, cost = O.remove_cost(F, n)
        D5, s5 = PC.remove(A, D, k, delta)
        D11, s11 = PC.remove_key(A, D, k, delta)
        assert np.array_equal(D5, want), (t, k)
        assert np.array_equal(D11, want), (t, k)
        assert (s5["phi"], s5["listed"]) == (phi, int(F.sum()))
        assert s5["cost"] == pytest.approx(cost)
        assert s5["fell_back"] == (cost > delta)
        assert s11["flagged"] == int(F.sum()) and s11["listed"] <= s11["flagged"] and s11["phi"] <= phi
        # the refined list keeps every pair whose distance changes
        keep = [x for x in range(n) if x != k]
        changed = int(O.refined_set(D[np.ix_(keep, keep)], want).sum())
        assert s11["listed"] >= changed


@pytest.mark.parametrize("delta", [0.0, 1.0])
def test_edge_equals_cold(delta):
    for t, A, und, rng in graphs():
        n = A.shape[0]
        if n < 2:
            continue
        D = O.fw(A)
        u, v = (int(x) for x in rng.choice(n, size=2, replace=False))
        for w in (0, 1, int(A[u, v]) if A[u, v] < INF else 5, int(rng.integers(1, 20000)), INF):
            A2, _ = O.apply_update(A, list(range(n)), "edge", u=u, v=v, w=w, undirected=und)
            Dn, st = PC.edge(A, D, u, v, w, delta, und)
            assert np.array_equal(Dn, O.fw(A2)), (t, u, v, w)
            assert st["removed"] in (u, v)


def test_query_paths_are_shortest():
    for t, A, und, rng in graphs():
        n = A.shape[0]
        D = O.fw(A)
        for _ in range(10):
            i, j = (int(x) for x in rng.integers(0, n, size=2))
            d, path, _ = PC.query(A, D, i, j)
            dc, pc, _ = PC.dijkstra_path(A, i, j)
            assert d == dc == int(D[i, j])
            for p in (path, pc):
                if D[i, j] >= INF:
                    assert p == []
                    continue
                assert p[0] == i and p[-1] == j
                assert sum(int(A[a, b]) for a, b in zip(p, p[1:])) == D[i, j]


def test_remove_sample_counts():
    """The benchmark's bounded sample reports Algorithm 5's Phi and list size
    and times at most the runs asked for."""
    A = W.random_graph(120, 1, 50, seed=3)
    D = O.fw(A)
    F = O.remove_mask(D, 7)
    s = PC.remove_sample(A, D, 7, 5)
    assert (s["phi"], s["listed"]) == (O.remove_cost(F, 120)[0], int(F.sum()))
    assert s["runs_timed"] == min(5, s["phi"]) and s["removal_s"] > 0
