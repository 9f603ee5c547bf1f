"""Warm-start all-pairs shortest paths on MI355X (gfx950).

The HIP library (libapsp.so, C ABI in include/apsp.h) keeps a dense graph's
APSP matrix on the GPU and updates it exactly after a node is added or
removed or an edge weight changes (arXiv 2412.15122).  `Graph` is the thin
Python face of that library; `workloads` holds the seeded synthetic inputs.

    from paper_2412_15122_amd import Graph
    g = Graph(adj, undirected=True, capacity=n + 100)   # cold start on cuda:0
    new_id = g.add_node(w_out)                          # weights to the live nodes, ascending ids
    g.remove_node(17)
    g.update_edge(3, 9, 250)                            # raise, lower or delete (INF)
    dist, path = g.query(3, 40)                         # warm single-pair path
    dist, on, key = g.query_nodes(3, 40)                # nodes on some / every shortest path
    D = g.matrix()                                      # ascending-id order

`Graph(..., minimax=True)` keeps minimax (bottleneck) distances instead.
`batch.Batch` runs many graphs' queued updates in one persistent launch and
`serve.Server` serves request streams over many resident graphs.
"""

__all__ = ["Graph", "INF"]

INF = 1 << 30


def __getattr__(name):
    if name == "Graph":
        from .apsp import Graph
        return Graph
    raise AttributeError(name)
