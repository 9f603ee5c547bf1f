"""CPU oracle for warm-start APSP -- TEST INFRASTRUCTURE ONLY.

Only `tests/`, `__graft_entry__.smoke()` and the benchmark's `cpu_baseline`
leg may import this module.  It shares no code with the HIP library and never
imports it.  Every routine here computes a *plain definition* from the paper,
slowly and visibly:

* ``fw`` / ``dijkstra_rows`` -- the cold APSP matrix (paper, Section 1;
  notation table: SPD with SPD(i,i) = 0 and the matrix M_G) by textbook
  Floyd-Warshall and dense Dijkstra, in C (``apsp_oracle.c``).
* ``brute_force_apsp`` / ``all_shortest_simple_paths`` -- enumeration of
  simple paths, straight from the definition of a path (the notation table's
  loop-free sequence Psi and the set Theta of all i->j paths); tiny n only.
* ``minimax_apsp`` / ``brute_force_minimax`` / ``minimax_by_thresholds`` --
  minimax (bottleneck) distances, the (min, max) variant of the discussion
  section: Floyd-Warshall with max, enumeration of simple paths, and
  reachability under a weight threshold.
* ``widest_apsp`` / ``brute_force_widest`` / ``widest_by_thresholds`` --
  widest (maximum-capacity) paths, the (max, min) variant the discussion
  section names beside minimax paths: Floyd-Warshall with min and max
  swapped, enumeration of simple paths, and reachability over edges of at
  least a given capacity.  W(i,i) = WIDEST_TOP (an empty walk is not
  limited), INF when j is unreachable.
* ``remove_mask`` -- the need_update_list of a node removal (Section 3.2,
  built with Theorem 4 / Corollary 3): pair (i,j)
  is listed when M[i][k] + M[k][j] equals M[i][j].
* ``remove_cost`` -- Definition 1: Phi / (N - 1).
* ``refined_set`` -- the refined need_update_list of Algorithms 11-12
  (Theorem 6): the pairs whose distance changes.
* ``edge_mask`` -- the same criterion applied to an edge (u,v): the pairs
  whose shortest distance can use the edge (see DESIGN for this reading).
* ``pair_nodes`` -- the nodes on some / on every shortest i -> j path
  (Algorithms 7, 8 and 10: candidate_node_list and key_node_list);
  ``minimax_pair_nodes`` the same over minimax paths.
* ``canonical_path`` -- the lexicographically smallest shortest simple path,
  taken greedily among Algorithm 7's candidates (correct when w >= 1).
* ``apply_update`` -- the updated graph G' of the notation table (G + p,
  G - G_k, or one edge re-weighted), as a plain adjacency edit.

All distances are int32 with INF = 2**30 and saturating sums computed in
int64 then clamped (the same value as the uint32 form of the C routines).
Matrices are in "compact" order: position a holds the a-th live id in
ascending order.
"""
from __future__ import annotations

import ctypes
import itertools
import os
import subprocess
from typing import List, Optional, Sequence, Tuple

import numpy as np

INF = 1 << 30

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "apsp_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (OpenMP).  Portable x86-64-v2 code so the
    library built here also runs on another host."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O3", "-march=x86-64-v2", "-fopenmp", "-shared",
                               "-fPIC", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        i32, p = ctypes.c_int32, ctypes.c_void_p
        lib.oracle_fw_init.argtypes = [i32, p, p]
        lib.oracle_fw_pivots.argtypes = [i32, p, i32, i32, ctypes.c_int]
        lib.oracle_dijkstra_rows.argtypes = [i32, p, p, i32, p, ctypes.c_int]
        lib.oracle_max_threads.argtypes = []
        for f in (lib.oracle_fw_init, lib.oracle_fw_pivots, lib.oracle_dijkstra_rows,
                  lib.oracle_max_threads):
            f.restype = ctypes.c_int
        _lib = lib
    return _lib


def max_threads() -> int:
    return int(_load().oracle_max_threads())


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _check_adj(A: np.ndarray) -> np.ndarray:
    A = np.ascontiguousarray(A, dtype=np.int32)
    assert A.ndim == 2 and A.shape[0] == A.shape[1]
    return A


def oplus(a, b):
    """Saturating concatenation a (+) b = min(a + b, INF) on int arrays."""
    return np.minimum(np.asarray(a, dtype=np.int64) + np.asarray(b, dtype=np.int64), INF)


# ---------------------------------------------------------------------------
# cold APSP
# ---------------------------------------------------------------------------

def fw_init(A: np.ndarray) -> np.ndarray:
    A = _check_adj(A)
    n = A.shape[0]
    D = np.empty_like(A)
    if _load().oracle_fw_init(n, _ptr(A), _ptr(D)) != 0:
        raise ValueError("adjacency weights must lie in [0, INF]")
    return D


def fw_pivots(D: np.ndarray, k0: int, k1: int, threads: int = 0) -> None:
    """Apply Floyd-Warshall pivots k0..k1-1 to D in place."""
    assert D.flags.c_contiguous and D.dtype == np.int32
    if _load().oracle_fw_pivots(D.shape[0], _ptr(D), k0, k1, threads) != 0:
        raise ValueError("bad pivot range")


def fw(A: np.ndarray, threads: int = 0) -> np.ndarray:
    """Cold APSP by textbook Floyd-Warshall."""
    D = fw_init(A)
    fw_pivots(D, 0, D.shape[0], threads)
    return D


def dijkstra_rows(A: np.ndarray, srcs: Sequence[int], threads: int = 0) -> np.ndarray:
    """Rows srcs of the APSP matrix, one dense Dijkstra per source."""
    A = _check_adj(A)
    s = np.ascontiguousarray(np.asarray(srcs, dtype=np.int32).reshape(-1))
    out = np.empty((s.size, A.shape[0]), dtype=np.int32)
    if _load().oracle_dijkstra_rows(A.shape[0], _ptr(A), _ptr(s), s.size, _ptr(out), threads) != 0:
        raise ValueError("bad source")
    return out


def dijkstra_cols(A: np.ndarray, dsts: Sequence[int], threads: int = 0) -> np.ndarray:
    """Columns dsts of the APSP matrix (Dijkstra on the reversed graph);
    result[r][i] = SPD(i, dsts[r])."""
    return dijkstra_rows(np.ascontiguousarray(np.asarray(A).T), dsts, threads)


# ---------------------------------------------------------------------------
# brute force (n <= 8): the definition of a path, enumerated
# ---------------------------------------------------------------------------

def _simple_paths(A: np.ndarray, i: int, j: int):
    """Every simple path i -> j over present edges, with its length."""
    n = A.shape[0]
    if i == j:
        yield (i,), 0
        return
    others = [t for t in range(n) if t != i and t != j]
    for r in range(len(others) + 1):
        for mid in itertools.permutations(others, r):
            seq = (i,) + mid + (j,)
            total = 0
            ok = True
            for a, b in zip(seq[:-1], seq[1:]):
                w = int(A[a, b])
                if w >= INF:
                    ok = False
                    break
                total += w
            if ok:
                yield seq, min(total, INF)


def brute_force_apsp(A: np.ndarray) -> np.ndarray:
    """SPD(i,j) = min over all simple i->j paths of the summed weight (INF if
    none), SPD(i,i) = 0."""
    A = _check_adj(A)
    n = A.shape[0]
    assert n <= 8, "brute force is for tiny graphs"
    D = np.full((n, n), INF, dtype=np.int64)
    for i in range(n):
        for j in range(n):
            for _, L in _simple_paths(A, i, j):
                D[i, j] = min(D[i, j], L)
    return D.astype(np.int32)


def all_shortest_simple_paths(A: np.ndarray, i: int, j: int) -> List[Tuple[int, ...]]:
    """All simple i->j paths of minimum length, lexicographically sorted."""
    A = _check_adj(A)
    paths = list(_simple_paths(A, i, j))
    if not paths:
        return []
    best = min(L for _, L in paths)
    if best >= INF:
        return []
    return sorted(p for p, L in paths if L == best)


# ---------------------------------------------------------------------------
# minimax (bottleneck) paths: the (min, max) semiring
# ---------------------------------------------------------------------------

def minimax_apsp(A: np.ndarray) -> np.ndarray:
    """Minimax distances: MM(i,j) = min over walks i -> j of the largest edge
    weight on the walk, MM(i,i) = 0, INF if j is unreachable -- the path
    problem the paper's discussion section names as a variant.  Textbook
    Floyd-Warshall with max in place of +, one numpy step per pivot."""
    D = _check_adj(A).astype(np.int64)
    n = D.shape[0]
    D[np.arange(n), np.arange(n)] = 0
    for k in range(n):
        D = np.minimum(D, np.maximum(D[:, k:k + 1], D[k:k + 1, :]))
    return D.astype(np.int32)


def minimax_rows(A: np.ndarray, srcs: Sequence[int]) -> np.ndarray:
    """Rows srcs of the minimax distance matrix by dense Dijkstra with max in
    place of + (a node's label is final once it is the least unsettled one,
    since max never lowers a label), one numpy step per settled node."""
    A = np.asarray(A)
    n = A.shape[0]
    out = np.empty((len(srcs), n), dtype=np.int32)
    for r, s in enumerate(srcs):
        dist = np.full(n, INF, dtype=np.int64)
        done = np.zeros(n, dtype=bool)
        dist[s] = 0
        for _ in range(n):
            cand = np.where(done, np.int64(INF) + 1, dist)
            u = int(np.argmin(cand))
            if cand[u] >= INF:
                break
            done[u] = True
            np.minimum(dist, np.maximum(dist[u], A[u].astype(np.int64)), out=dist, where=~done)
        out[r] = dist
    return out


def brute_force_minimax(A: np.ndarray) -> np.ndarray:
    """MM(i,j) = min over all simple i->j paths of the largest edge weight
    (a walk's cycles can be cut without raising its largest edge), n <= 8."""
    A = _check_adj(A)
    n = A.shape[0]
    assert n <= 8, "brute force is for tiny graphs"
    D = np.full((n, n), INF, dtype=np.int64)
    for i in range(n):
        for j in range(n):
            for seq, L in _simple_paths(A, i, j):
                if L >= INF:
                    continue
                D[i, j] = min(D[i, j], max((int(A[a, b]) for a, b in zip(seq[:-1], seq[1:])), default=0))
    return D.astype(np.int32)


def minimax_by_thresholds(A: np.ndarray) -> np.ndarray:
    """MM(i,j) as the least threshold theta (0 or an edge weight) at which j
    is reachable from i over edges of weight <= theta: reachability by
    breadth-first search, one threshold at a time."""
    A = _check_adj(A).astype(np.int64)
    n = A.shape[0]
    D = np.full((n, n), INF, dtype=np.int64)
    levels = sorted({0} | {int(w) for w in A[A < INF]})
    for theta in reversed(levels):
        adj = (A <= theta)
        for i in range(n):
            seen = np.zeros(n, dtype=bool)
            seen[i] = True
            frontier = [i]
            while frontier:
                nxt = np.nonzero(adj[frontier].any(axis=0) & ~seen)[0]
                seen[nxt] = True
                frontier = list(nxt)
            D[i, seen] = theta
    return D.astype(np.int32)


# ---------------------------------------------------------------------------
# widest (maximum-capacity) paths: the (max, min) semiring
# ---------------------------------------------------------------------------

WIDEST_TOP = INF - 1   # the largest capacity; the width of the empty walk i -> i


def widest_apsp(C: np.ndarray) -> np.ndarray:
    """Widest-path widths: W(i,j) = max over walks i -> j of the smallest
    edge capacity on the walk, W(i,i) = WIDEST_TOP, INF if j is unreachable.
    Capacities in [0, WIDEST_TOP], INF = no edge.  Textbook Floyd-Warshall
    with (max, min) in place of (min, +); 'no path' is -1 inside."""
    C = _check_adj(C).astype(np.int64)
    n = C.shape[0]
    W = np.where(C >= INF, -1, C)
    W[np.arange(n), np.arange(n)] = WIDEST_TOP
    for k in range(n):
        W = np.maximum(W, np.minimum(W[:, k:k + 1], W[k:k + 1, :]))
    return np.where(W < 0, INF, W).astype(np.int32)


def brute_force_widest(C: np.ndarray) -> np.ndarray:
    """W(i,j) = max over all simple i -> j paths of the smallest capacity
    (cutting a cycle out of a walk never lowers its smallest capacity),
    n <= 8."""
    C = _check_adj(C)
    n = C.shape[0]
    assert n <= 8, "brute force is for tiny graphs"
    W = np.full((n, n), -1, dtype=np.int64)
    for i in range(n):
        W[i, i] = WIDEST_TOP
        for j in range(n):
            if i == j:
                continue
            for seq, _ in _simple_paths(C, i, j):   # every edge of seq is present
                W[i, j] = max(W[i, j], min(int(C[a, b]) for a, b in zip(seq[:-1], seq[1:])))
    return np.where(W < 0, INF, W).astype(np.int32)


def widest_by_thresholds(C: np.ndarray) -> np.ndarray:
    """W(i,j) as the largest threshold t (an edge capacity) at which j is
    reachable from i over edges of capacity >= t: breadth-first search, one
    threshold at a time from the largest down."""
    C = _check_adj(C).astype(np.int64)
    n = C.shape[0]
    W = np.full((n, n), INF, dtype=np.int64)
    done = np.eye(n, dtype=bool)
    W[np.arange(n), np.arange(n)] = WIDEST_TOP
    for t in sorted({int(c) for c in C[C < INF]}, reverse=True):
        adj = (C >= t) & (C < INF)
        for i in range(n):
            seen = np.zeros(n, dtype=bool)
            seen[i] = True
            frontier = [i]
            while frontier:
                nxt = np.nonzero(adj[frontier].any(axis=0) & ~seen)[0]
                seen[nxt] = True
                frontier = list(nxt)
            new = seen & ~done[i]
            W[i, new] = t
            done[i] |= seen
    return W.astype(np.int32)


# ---------------------------------------------------------------------------
# masks, cost, query
# ---------------------------------------------------------------------------

def remove_mask(D: np.ndarray, k: int, minimax: bool = False) -> np.ndarray:
    """need_update_list of removing compact node k, as a boolean matrix:
    F[i][j] is True when i != j, k not in {i, j}, D[i][j] < INF and
    D[i][k] (+) D[k][j] == D[i][j]  (equality form of Corollary 3;
    for distances '>=' and '==' coincide).  minimax: (+) is max."""
    D = np.asarray(D, dtype=np.int64)
    n = D.shape[0]
    cat = np.maximum if minimax else oplus
    F = (cat(D[:, k][:, None], D[k, :][None, :]) == D) & (D < INF)
    F[np.arange(n), np.arange(n)] = False
    F[k, :] = False
    F[:, k] = False
    return F


def remove_cost(F: np.ndarray, n_before: int) -> Tuple[int, float]:
    """Definition 1: Phi = number of non-empty need_update_list
    rows, Cost = Phi / (N - 1) with N the node count before the removal."""
    phi = int(np.count_nonzero(F.any(axis=1)))
    cost = 0.0 if n_before <= 1 else phi / (n_before - 1)
    return phi, cost


def edge_mask(D: np.ndarray, u: int, v: int, w_old: int, undirected: bool, minimax: bool = False) -> np.ndarray:
    """Pairs whose shortest distance can use edge u->v of weight w_old:
    i != j, D[i][j] < INF and D[i][u] (+) w_old (+) D[v][j] == D[i][j]; for an
    undirected graph also the v->u direction.  minimax: (+) is max."""
    D = np.asarray(D, dtype=np.int64)
    n = D.shape[0]
    cat = np.maximum if minimax else oplus
    F = cat(cat(D[:, u][:, None], w_old), D[v, :][None, :]) == D
    if undirected:
        F |= cat(cat(D[:, v][:, None], w_old), D[u, :][None, :]) == D
    F &= D < INF
    F[np.arange(n), np.arange(n)] = False
    return F


def refined_set(D_before: np.ndarray, D_after: np.ndarray) -> np.ndarray:
    """The refined need_update_list of Algorithms 11 and 12: the pairs whose
    shortest distance differs between G and G' (both matrices over the same
    nodes in the same order; for a removal, pass D_before without row and
    column k).  By Theorem 6 a pair whose distance goes up had k
    (or the raised edge) on every shortest path, and a pair with a shortest
    path avoiding it keeps its distance, so this is the paper's refined list."""
    return np.asarray(D_before, dtype=np.int64) != np.asarray(D_after, dtype=np.int64)


def edge_scope(col_u, col_v, row_u, row_v, w: int) -> Tuple[int, int]:
    """|R| and |C| of edge u->v with weight w, from column u, column v, row u and
    row v of the APSP matrix: R = {i: D[i][u] (+) w == D[i][v] < INF},
    C = {j: w (+) D[v][j] == D[u][j] < INF}.  |R|*|C| bounds the number of pairs
    whose shortest path the edge can carry."""
    col_u, col_v = np.asarray(col_u, np.int64), np.asarray(col_v, np.int64)
    row_u, row_v = np.asarray(row_u, np.int64), np.asarray(row_v, np.int64)
    R = int(np.count_nonzero((oplus(col_u, w) == col_v) & (col_v < INF)))
    C = int(np.count_nonzero((oplus(w, row_v) == row_u) & (row_u < INF)))
    return R, C


def canonical_path(A: np.ndarray, D: np.ndarray, i: int, j: int) -> List[int]:
    """Lexicographically smallest shortest simple i->j path (compact indices).

    Candidates are Algorithm 7's: t with D[i][t] (+) D[t][j] == D[i][j]
    (Theorem 5: they contain every shortest path).  From cur, the
    next node is the smallest b != cur with A[cur][b] < INF and
    A[cur][b] (+) D[b][j] == D[cur][j].  With w >= 1 each step lowers
    D[.][j], so the walk is simple and ends at j.  Returns [] if unreachable.
    """
    A = np.asarray(A, dtype=np.int64)
    D = np.asarray(D, dtype=np.int64)
    if i == j:
        return [i]
    if D[i, j] >= INF:
        return []
    n = D.shape[0]
    cand = [t for t in range(n) if t in (i, j) or oplus(D[i, t], D[t, j]) == D[i, j]]
    path = [i]
    cur = i
    while cur != j:
        nxt = None
        for b in cand:  # ascending
            if b == cur or A[cur, b] >= INF:
                continue
            if oplus(A[cur, b], D[b, j]) == D[cur, j]:
                nxt = b
                break
        if nxt is None or len(path) > n:
            raise RuntimeError("no canonical successor (zero-weight cycle?)")
        path.append(nxt)
        cur = nxt
    return path


# ---------------------------------------------------------------------------
# the updated graph G'
# ---------------------------------------------------------------------------

def pair_nodes(A: np.ndarray, D: np.ndarray, i: int, j: int) -> Tuple[List[int], List[int]]:
    """The nodes of the shortest i -> j paths, in compact positions, ascending.

    on  -- Algorithm 7's candidate_node_list (Theorem 5), which is
           the node set of Algorithm 8's paths: every t with
           D[i][t] (+) D[t][j] == D[i][j], i and j included.
    key -- Algorithm 10's key_node_list of the pair: the nodes other than i
           and j that every shortest i -> j walk visits.  Written out by its
           definition: t is one when j cannot be reached from i over tight
           edges (x -> y with D[i][x] (+) A[x][y] == D[i][y], both on) once t
           is taken out -- a walk over tight edges from i to j has length
           D[i][j], and every shortest walk is one.
    i == j gives ([i], []); an unreachable pair ([], []).  Only row i and
    column j of D are read (``pair_nodes_from``)."""
    D = np.asarray(D)
    return pair_nodes_from(A, D[i, :], D[:, j], i, j)


def pair_nodes_from(A: np.ndarray, di, dj, i: int, j: int) -> Tuple[List[int], List[int]]:
    """``pair_nodes`` given di[t] = D[i][t] and dj[t] = D[t][j] (e.g. one
    Dijkstra row from i and one column into j on a large graph); A is read
    entry by entry."""
    A = np.asarray(A)
    di = np.asarray(di, dtype=np.int64)
    dj = np.asarray(dj, dtype=np.int64)
    if i == j:
        return [i], []
    d = int(di[j])
    if d >= INF:
        return [], []
    on = [int(t) for t in np.nonzero(oplus(di, dj) == d)[0]]
    on_set = set(on)

    def reaches_without(t):
        seen = {i}
        stack = [i]
        while stack:
            x = stack.pop()
            if x == j:
                return True
            for y in on:
                if y in seen or y == t or y == x:
                    continue
                w = int(A[x, y])
                if w < INF and int(di[x]) + w == int(di[y]):
                    seen.add(y)
                    stack.append(y)
        return False

    key = [t for t in on if t != i and t != j and not reaches_without(t)]
    assert i in on_set and j in on_set
    return on, key


def minimax_pair_nodes(A: np.ndarray, D: np.ndarray, i: int, j: int) -> Tuple[List[int], List[int]]:
    """``pair_nodes`` over minimax paths (D the minimax matrix): the nodes on
    some optimal i -> j walk, t with max(D[i][t], D[t][j]) == D[i][j], and
    the nodes other than i and j on every one.  An optimal walk is any walk
    whose edges all weigh at most d = D[i][j] (its largest edge is then d),
    so t is a key node when j cannot be reached from i over edges <= d once
    t is taken out."""
    D = np.asarray(D)
    return minimax_pair_nodes_from(A, D[i, :], D[:, j], i, j)


def minimax_key_test(A: np.ndarray, i: int, j: int, d: int, t: int) -> bool:
    """Is t on every walk from i to j over edges of weight <= d?"""
    light = np.asarray(A) <= d
    seen = np.zeros(light.shape[0], dtype=bool)
    seen[i] = seen[t] = True
    frontier = [i]
    while frontier and not seen[j]:
        nxt = np.nonzero(light[frontier].any(axis=0) & ~seen)[0]
        seen[nxt] = True
        frontier = list(nxt)
    return not bool(seen[j])


def minimax_pair_nodes_from(A: np.ndarray, di, dj, i: int, j: int) -> Tuple[List[int], List[int]]:
    """``minimax_pair_nodes`` given di[t] = D[i][t] and dj[t] = D[t][j]."""
    A = np.asarray(A)
    di = np.asarray(di, dtype=np.int64)
    dj = np.asarray(dj, dtype=np.int64)
    if i == j:
        return [i], []
    d = int(di[j])
    if d >= INF:
        return [], []
    on = [int(t) for t in np.nonzero(np.maximum(di, dj) == d)[0]]
    light = A <= d

    def reaches_without(t):
        seen = np.zeros(A.shape[0], dtype=bool)
        seen[i] = seen[t] = True
        frontier = [i]
        while frontier:
            if seen[j] and j != t:
                return True
            nxt = np.nonzero(light[frontier].any(axis=0) & ~seen)[0]
            seen[nxt] = True
            frontier = list(nxt)
        return bool(seen[j])

    key = [t for t in on if t != i and t != j and not reaches_without(t)]
    return on, key


def apply_update(A: np.ndarray, ids: List[int], kind: str, *, u: int = -1, v: int = -1,
                 w: int = 0, w_out=None, w_in=None, undirected: bool = False):
    """Return (A', ids') for one update, in compact ascending-id order.

    add:      G + p -- p gets id max(ids)+1 (or 0), appended last; row p is
              w_out, column p is w_in (w_in = w_out if undirected).
    remove:   G - G_k -- row and column of id u deleted.
    edge:     (kinds 'decrease' / 'increase' / 'edge') weight of u->v set to
              w (and v->u if undirected).
    """
    A = np.asarray(A, dtype=np.int32)
    n = A.shape[0]
    if kind == "add":
        w_out = np.asarray(w_out, dtype=np.int32).reshape(n)
        w_in = w_out if (w_in is None or undirected) else np.asarray(w_in, dtype=np.int32).reshape(n)
        B = np.empty((n + 1, n + 1), dtype=np.int32)
        B[:n, :n] = A
        B[n, :n] = w_out
        B[:n, n] = w_in
        B[n, n] = 0
        return B, list(ids) + [(max(ids) + 1) if ids else 0]
    if kind == "remove":
        a = ids.index(u)
        keep = [x for x in range(n) if x != a]
        return np.ascontiguousarray(A[np.ix_(keep, keep)]), [x for x in ids if x != u]
    if kind in ("decrease", "increase", "edge"):
        a, b = ids.index(u), ids.index(v)
        B = A.copy()
        B[a, b] = w
        if undirected:
            B[b, a] = w
        return B, list(ids)
    raise ValueError(kind)
