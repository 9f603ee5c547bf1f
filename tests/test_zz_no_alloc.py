"""The edge update that allocates nothing (apsp_update_edge_noalloc) against
apsp_update_edge, through the C ABI.

Two graphs in a row, the second smaller, each with a clone: every edge
update (tight increases with many flagged rows, decreases, no-ops, a
deletion and an insertion) goes to the graph through the no-allocation call
and to its clone through apsp_update_edge; D, A, ids and the update
statistics must be equal after every update, and the final matrices equal
the oracle's Floyd-Warshall.  A graph above the size limit is refused with
nothing changed.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2412_15122_amd import workloads as W

pytestmark = pytest.mark.gpu

INF = W.INF


def log(*a):
    print(*a, flush=True)


def edge_plan(rng, A, D, undirected, count):
    """Edge updates on the current graph: tight increases first (the edge is a
    shortest path between its ends, so pairs are flagged), then a mix."""
    n = A.shape[0]
    tight = [(u, v) for u in range(n) for v in range(n)
             if u != v and A[u, v] < INF and A[u, v] == D[u, v]]
    plan = []
    for t in range(count):
        if t % 3 == 0 and tight:
            u, v = tight[int(rng.integers(len(tight)))]
            plan.append((u, v, int(A[u, v]) + int(rng.integers(1, 6))))
        elif t % 3 == 1:
            u, v = (int(x) for x in rng.choice(n, size=2, replace=False))
            plan.append((u, v, int(rng.integers(0, 3))))          # usually a decrease
        else:
            u, v = (int(x) for x in rng.choice(n, size=2, replace=False))
            plan.append((u, v, int(rng.integers(1, 12))))
    u, v = (int(x) for x in rng.choice(n, size=2, replace=False))
    plan.append((u, v, INF))                                      # deletion
    plan.append((u, v, 3))                                        # insertion back
    return plan


def run_case(n, undirected, seed, policy=None):
    import torch
    from paper_2412_15122_amd.apsp import Graph
    rng = np.random.default_rng(seed)
    A = W.random_graph(n, 1, 6, undirected=undirected, density=0.6, seed=seed)   # small weights: ties
    g = Graph(A, undirected=undirected, capacity=n + 9)
    h = g.clone()
    if policy is not None:
        g.set_fallback(*policy)
        h.set_fallback(*policy)
    ids = list(range(n))
    D = O.fw(A)
    plan = edge_plan(rng, A, D, undirected, 24)
    heavy = 0
    for t, (u, v, w) in enumerate(plan):
        g.update_edge_noalloc(u, v, w)
        h.update_edge(u, v, w)
        sg, sh = g.stats(), h.stats()
        assert sg == sh, (t, u, v, w, sg, sh)
        heavy += sg["heavy_rows"] > 0
        assert torch.equal(g.matrix_device("D"), h.matrix_device("D")), (t, u, v, w)
        assert torch.equal(g.matrix_device("A"), h.matrix_device("A")), (t, u, v, w)
        A, ids = O.apply_update(A, ids, "edge", u=u, v=v, w=w, undirected=undirected)
    assert g.ids() == h.ids() == ids
    assert np.array_equal(g.matrix(), O.fw(A))
    log(f"n={n} undirected={undirected}: {len(plan)} updates equal, {heavy} with heavy rows")
    g.sync()
    h.sync()
    g.close()
    h.close()
    return heavy


def test_noalloc_edge_updates_equal_the_allocating_call_two_graphs():
    heavy = run_case(300, False, 11)          # first call on the device: the scratch lookup
    heavy += run_case(90, True, 12)           # second, smaller graph over the same array
    assert heavy > 0                          # the heavy-row pass ran through the static scratch


def test_noalloc_with_the_cost_fallback():
    run_case(140, False, 13, policy=(1, 0.0))  # every flagged increase runs the cold recompute


def test_noalloc_refuses_a_graph_above_the_limit():
    import torch
    from paper_2412_15122_amd import _native as N
    from paper_2412_15122_amd.apsp import Graph
    n = 40
    A = W.random_graph(n, 1, 50, seed=5)
    g = Graph(A, capacity=N.APSP_NOALLOC_MAX_CAPACITY + 1)
    D0 = g.matrix_device("D").clone()
    with pytest.raises(N.ApspError) as e:
        g.update_edge_noalloc(0, 1, 1)
    assert "APSP_NOALLOC_MAX_CAPACITY" in str(e.value)
    assert torch.equal(g.matrix_device("D"), D0)
    g.update_edge(0, 1, 1)                    # the allocating call still takes it
    A2, _ = O.apply_update(A, list(range(n)), "edge", u=0, v=1, w=1)
    assert np.array_equal(g.matrix(), O.fw(A2))
    g.close()
