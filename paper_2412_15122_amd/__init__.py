"""Warm-start all-pairs shortest paths on MI355X (gfx950).

The HIP library (libapsp.so, C ABI in include/apsp.h) keeps a dense graph's
APSP matrix on the GPU and updates it exactly after a node is added or
removed or an edge weight changes (arXiv 2412.15122).  `Graph` is the thin
Python face of that library; `workloads` holds the seeded synthetic inputs.
"""

__all__ = ["Graph", "INF"]

INF = 1 << 30


def __getattr__(name):
    if name == "Graph":
        from .apsp import Graph
        return Graph
    raise AttributeError(name)
