"""Seeded synthetic inputs: dense weighted graphs and update streams.

This module only draws random numbers and keeps the bookkeeping an update
stream needs (which ids are live, what weight an edge has now).  It holds
none of the shortest-path arithmetic: it never computes a distance, a mask
or a relaxation, so both the HIP path and the CPU oracle can consume its
arrays without sharing any of the method's code.

Graph model (paper, Section 1 and the notation table): a dense directed graph
with non-negative integer edge weights; an undirected graph is the symmetric
special case.  Weights are int32; an absent edge carries the sentinel
INF = 2**30.  The diagonal is 0.

Ids follow the paper's G+p / G-G_k semantics (notation table): the n nodes of
a fresh graph have ids 0..n-1, an added node gets id max_id+1, and a removed
id never comes back.  Every vector indexed by node (an added node's out- and
in-weights) is in ascending-id order.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Optional, Tuple

import numpy as np

INF = 1 << 30

ADD, REMOVE, DECREASE, INCREASE = "add", "remove", "decrease", "increase"
# edge updates that cross INF: an existing edge removed (its weight set to INF)
# and an absent edge inserted with a finite weight
DELETE, INSERT = "delete", "insert"

_SEED_BASE = 2412151220


def seed_for(config: int) -> int:
    """Seed of workload `config` (1..5)."""
    return _SEED_BASE + int(config)


# ---------------------------------------------------------------------------
# graphs
# ---------------------------------------------------------------------------

def random_graph(n: int, wmin: int, wmax: int, *, undirected: bool = False,
                 density: float = 1.0, seed=0,
                 zero_frac: float = 0.0) -> np.ndarray:
    """Dense adjacency matrix, int32 (n, n), diagonal 0, absent edge = INF.

    Each ordered pair i != j carries an edge with probability `density`
    (independently; for undirected graphs per unordered pair), with a weight
    uniform on [wmin, wmax].  `zero_frac` turns that fraction of present
    edges into zero-weight edges (the paper allows w >= 0).
    """
    rng = np.random.default_rng(seed)
    a = rng.integers(wmin, wmax + 1, size=(n, n), dtype=np.int32)
    if zero_frac > 0.0:
        a[rng.random((n, n)) < zero_frac] = 0
    if density < 1.0:
        a[rng.random((n, n)) >= density] = INF
    if undirected:
        a = np.triu(a, 1)
        a = a + a.T
    np.fill_diagonal(a, 0)
    return np.ascontiguousarray(a, dtype=np.int32)


def symmetric_complete_graph(n: int, wmin: int, wmax: int, seed) -> np.ndarray:
    """Undirected complete graph with symmetric uniform weights: the upper
    triangle is drawn, the lower one mirrors it block by block (so n = 16384,
    1 GiB, needs little more than one matrix of host memory)."""
    rng = np.random.default_rng(seed)
    a = rng.integers(wmin, wmax + 1, size=(n, n), dtype=np.int32)
    blk = 2048
    for r0 in range(0, n, blk):
        r1 = min(n, r0 + blk)
        d = a[r0:r1, r0:r1]
        low = np.tril_indices(r1 - r0, -1)
        d[low] = d.T[low]
        for c0 in range(0, r0, blk):
            c1 = min(n, c0 + blk)
            a[r0:r1, c0:c1] = a[c0:c1, r0:r1].T
    np.fill_diagonal(a, 0)
    return a


# ---------------------------------------------------------------------------
# update streams
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class Update:
    """One update of the stream.

    kind      ADD | REMOVE | DECREASE | INCREASE | DELETE | INSERT
    u, v      edge endpoints (ids) for edge updates; u = id for REMOVE
    w         new edge weight for edge updates
    old       weight of the edge before the update (edge updates)
    w_out     ADD: weights new->t for every live t, ascending-id order
    w_in      ADD: weights t->new (same order); equals w_out if undirected
    new_id    ADD: the id the node receives (max_id + 1)
    """
    kind: str
    u: int = -1
    v: int = -1
    w: int = 0
    old: int = 0
    w_out: Optional[np.ndarray] = None
    w_in: Optional[np.ndarray] = None
    new_id: int = -1


class GraphState:
    """Host bookkeeping of a graph under updates: live ids and current weights.

    The base matrix is kept as generated; later changes sit in small
    overlays, so that a 1 GiB base never has to be copied.  `weight(u, v)`
    returns the current weight of edge u->v (INF if absent).
    """

    def __init__(self, adj: np.ndarray, undirected: bool):
        self.base = adj
        self.n0 = adj.shape[0]
        self.undirected = undirected
        self.live: List[int] = list(range(self.n0))
        self.max_id = self.n0 - 1
        self.edits: Dict[Tuple[int, int], int] = {}
        # added node id -> (ids live when it was added (ascending), out-weights, in-weights)
        self.added: Dict[int, Tuple[np.ndarray, np.ndarray, np.ndarray]] = {}

    def _added_weight(self, node: int, other: int, out: bool) -> Optional[int]:
        rec = self.added.get(node)
        if rec is None:
            return None
        ids, w_out, w_in = rec
        pos = int(np.searchsorted(ids, other))
        if pos < ids.size and ids[pos] == other:
            return int((w_out if out else w_in)[pos])
        return None

    def weight(self, u: int, v: int) -> int:
        if u == v:
            return 0
        key = (u, v)
        if key in self.edits:
            return self.edits[key]
        # an edge touching an added node was drawn when the younger endpoint
        # was added: it sits in that node's out- or in-weights
        w = self._added_weight(u, v, True)
        if w is None:
            w = self._added_weight(v, u, False)
        if w is None:
            w = int(self.base[u, v])
        return w

    def set_weight(self, u: int, v: int, w: int) -> None:
        self.edits[(u, v)] = int(w)
        if self.undirected:
            self.edits[(v, u)] = int(w)

    def add(self, w_out: np.ndarray, w_in: np.ndarray) -> int:
        nid = self.max_id + 1
        self.max_id = nid
        self.added[nid] = (np.asarray(self.live, dtype=np.int64), np.asarray(w_out), np.asarray(w_in))
        self.live.append(nid)
        return nid

    def remove(self, k: int) -> None:
        self.live.remove(k)

    def dense(self) -> np.ndarray:
        """Current adjacency in ascending-id order (small graphs only)."""
        ids = self.live
        n = len(ids)
        out = np.empty((n, n), dtype=np.int32)
        for a, i in enumerate(ids):
            for b, j in enumerate(ids):
                out[a, b] = self.weight(i, j)
        return out


def _pick_edge(rng, st: GraphState) -> Tuple[int, int, int]:
    """A random existing edge u->v (u != v) between live nodes."""
    for _ in range(10000):
        u, v = rng.choice(len(st.live), size=2, replace=False)
        u, v = st.live[int(u)], st.live[int(v)]
        w = st.weight(u, v)
        if w < INF:
            return u, v, w
    raise RuntimeError("no edge found")


def _pick_absent_edge(rng, st: GraphState) -> Tuple[int, int]:
    """A random absent edge u->v (u != v, weight INF) between live nodes."""
    for _ in range(10000):
        u, v = rng.choice(len(st.live), size=2, replace=False)
        u, v = st.live[int(u)], st.live[int(v)]
        if st.weight(u, v) >= INF:
            return u, v
    raise RuntimeError("no absent edge found")


def _draw_weights(rng, m: int, wmin: int, wmax: int, density: float) -> np.ndarray:
    w = rng.integers(wmin, wmax + 1, size=m, dtype=np.int32)
    if density < 1.0:
        w[rng.random(m) >= density] = INF
    return w


def make_update(rng, st: GraphState, kind: str, *, wmin: int, wmax: int,
                inc_max: int, density: float = 1.0) -> Update:
    """Draw one update of `kind` against the current state and apply it to the
    bookkeeping.  Decrease: new weight uniform on [1, old] (0 stays 0); increase: uniform on
    [old, max(old, inc_max)]; delete: an existing edge set to INF; insert: an
    absent edge given a weight uniform on [wmin, wmax]."""
    if kind == ADD:
        m = len(st.live)
        w_out = _draw_weights(rng, m, wmin, wmax, density)
        w_in = w_out.copy() if st.undirected else _draw_weights(rng, m, wmin, wmax, density)
        nid = st.add(w_out, w_in)
        return Update(ADD, w_out=w_out, w_in=w_in, new_id=nid)
    if kind == REMOVE:
        k = st.live[int(rng.integers(0, len(st.live)))]
        st.remove(k)
        return Update(REMOVE, u=k)
    if kind == INSERT:
        u, v = _pick_absent_edge(rng, st)
        w = int(rng.integers(wmin, wmax + 1))
        st.set_weight(u, v, w)
        return Update(kind, u=u, v=v, w=w, old=INF)
    u, v, old = _pick_edge(rng, st)
    if kind == DELETE:
        w = INF
    elif kind == DECREASE:
        w = int(rng.integers(min(1, old), old + 1))   # a zero-weight edge stays 0
    elif kind == INCREASE:
        w = int(rng.integers(old, max(old, inc_max) + 1))
    else:
        raise ValueError(kind)
    st.set_weight(u, v, w)
    return Update(kind, u=u, v=v, w=w, old=old)


def kinds_shuffled(rng, counts: Dict[str, int]) -> List[str]:
    ks: List[str] = []
    for k in (ADD, REMOVE, DECREASE, INCREASE):
        ks += [k] * counts.get(k, 0)
    perm = rng.permutation(len(ks))
    return [ks[i] for i in perm]


# ---------------------------------------------------------------------------
# the five workloads
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class Workload:
    name: str
    adj: np.ndarray
    undirected: bool
    updates: List[Update]
    wmin: int
    wmax: int
    inc_max: int
    density: float = 1.0


def config1(seed: Optional[int] = None) -> Workload:
    """Directed complete graph, n = 256, weights U[1, 1000]; one update of each
    kind in the order add, remove, decrease (to U[1, old]), increase (to
    U[old, 2000])."""
    ss = np.random.SeedSequence(seed_for(1) if seed is None else seed)
    g_seed, u_seed = ss.spawn(2)
    adj = random_graph(256, 1, 1000, seed=g_seed)
    st = GraphState(adj, False)
    rng = np.random.default_rng(u_seed)
    ups = [make_update(rng, st, k, wmin=1, wmax=1000, inc_max=2000)
           for k in (ADD, REMOVE, DECREASE, INCREASE)]
    return Workload("directed complete n=256 U[1,1000]", adj, False, ups, 1, 1000, 2000)


def config2(seed: Optional[int] = None, n: int = 4096) -> Workload:
    """Directed graph, n = 4096, each ordered pair present with probability 0.95,
    weights U[1, 10000]; one update of each kind."""
    ss = np.random.SeedSequence(seed_for(2) if seed is None else seed)
    g_seed, u_seed = ss.spawn(2)
    adj = random_graph(n, 1, 10000, density=0.95, seed=g_seed)
    st = GraphState(adj, False)
    rng = np.random.default_rng(u_seed)
    ups = [make_update(rng, st, k, wmin=1, wmax=10000, inc_max=20000, density=0.95)
           for k in (ADD, REMOVE, DECREASE, INCREASE)]
    return Workload(f"directed n={n} density 0.95 U[1,10000]", adj, False, ups,
                    1, 10000, 20000, 0.95)


CFG3_COUNTS = {ADD: 300, REMOVE: 200, DECREASE: 250, INCREASE: 250}


def config3_graph(n: int = 16384, seed: Optional[int] = None) -> np.ndarray:
    """Undirected complete graph with symmetric weights U[1, 10000]."""
    ss = np.random.SeedSequence(seed_for(3) if seed is None else seed)
    g_seed = ss.spawn(1)[0]
    return symmetric_complete_graph(n, 1, 10000, g_seed)


class Config3Stream:
    """The seeded update stream on the undirected complete graph: blocks of
    1000 updates with exact counts 300 add / 200 remove / 250 decrease /
    250 increase in a seeded shuffle.  Add: symmetric weights U[1, 10000];
    decrease U[1, old]; increase U[old, 20000].  The block's worst-case
    increase is supplied by the caller (it depends on distances) and is
    placed first; it counts as one of the 250 increases."""

    def __init__(self, adj: np.ndarray, seed: Optional[int] = None,
                 counts: Optional[Dict[str, int]] = None):
        ss = np.random.SeedSequence(seed_for(3) if seed is None else seed)
        _, u_seed = ss.spawn(2)
        self.rng = np.random.default_rng(u_seed)
        self.state = GraphState(adj, True)
        self.counts = dict(CFG3_COUNTS if counts is None else counts)

    def next_block(self, worst: Optional[Tuple[int, int, int]] = None) -> List[Update]:
        counts = dict(self.counts)
        ups: List[Update] = []
        if worst is not None:
            u, v, w_new = worst
            old = self.state.weight(u, v)
            self.state.set_weight(u, v, w_new)
            ups.append(Update(INCREASE, u=u, v=v, w=w_new, old=old))
            counts[INCREASE] -= 1
        for k in kinds_shuffled(self.rng, counts):
            ups.append(make_update(self.rng, self.state, k, wmin=1, wmax=10000,
                                   inc_max=20000))
        return ups


def lightest_edges(adj: np.ndarray, m: int, undirected: bool) -> List[Tuple[int, int, int]]:
    """The m lightest present edges (u, v, w) of a dense adjacency, ties broken
    by lowest (u, v); for undirected graphs only u < v is listed.  Used to
    shortlist the candidates of the worst-case increase."""
    n = adj.shape[0]
    blk = max(1, (1 << 24) // max(n, 1))

    def entries(limit):
        out = []
        for r0 in range(0, n, blk):
            b = adj[r0:r0 + blk]
            rows, cols = np.nonzero(b <= limit)
            for r, c in zip(rows.tolist(), cols.tolist()):
                u = r0 + r
                if u == c or (undirected and u > c):
                    continue
                out.append((int(b[r, c]), u, c))
        return out

    limit = 1
    while True:
        found = entries(limit)
        if len(found) >= m or limit >= INF - 1:
            break
        limit = min(INF - 1, limit * 2)
    found.sort()
    return [(u, v, w) for (w, u, v) in found[:m]]


def config4(seed: Optional[int] = None, graphs: int = 512, updates_per_graph: int = 8):
    """Many independent directed complete graphs, n = round(exp(U(ln 128,
    ln 2048))), weights U[1, 5000], each with `updates_per_graph` queued
    updates whose kinds are drawn 30/20/25/25 (add/remove/decrease/increase);
    decrease U[1, old], increase U[old, 10000]."""
    ss = np.random.SeedSequence(seed_for(4) if seed is None else seed)
    n_seed, g_seed, u_seed = ss.spawn(3)
    rng_n = np.random.default_rng(n_seed)
    ns = np.rint(np.exp(rng_n.uniform(math.log(128), math.log(2048), size=graphs))).astype(int)
    g_seeds = g_seed.spawn(graphs)
    u_seeds = u_seed.spawn(graphs)
    out = []
    p = [0.30, 0.20, 0.25, 0.25]
    for gi in range(graphs):
        adj = random_graph(int(ns[gi]), 1, 5000, seed=g_seeds[gi])
        st = GraphState(adj, False)
        rng = np.random.default_rng(u_seeds[gi])
        kinds = [(ADD, REMOVE, DECREASE, INCREASE)[int(i)]
                 for i in rng.choice(4, size=updates_per_graph, p=p)]
        ups = [make_update(rng, st, k, wmin=1, wmax=5000, inc_max=10000) for k in kinds]
        out.append(Workload(f"batched graph {gi} n={ns[gi]}", adj, False, ups, 1, 5000, 10000))
    return out


QUERY = "query"
SERVE_MIX = [(INCREASE, 0.45), (DECREASE, 0.45), (ADD, 0.025), (REMOVE, 0.025), (QUERY, 0.05)]


def config5_graphs(seed: Optional[int] = None, graphs: int = 64,
                   nmin: int = 1024, nmax: int = 8192):
    """Resident directed complete graphs, n uniform on [nmin, nmax], weights
    U[1, 10000]."""
    ss = np.random.SeedSequence(seed_for(5) if seed is None else seed)
    n_seed, g_seed, _ = ss.spawn(3)
    ns = np.random.default_rng(n_seed).integers(nmin, nmax + 1, size=graphs)
    g_seeds = g_seed.spawn(graphs)
    return [random_graph(int(ns[g]), 1, 10000, seed=g_seeds[g]) for g in range(graphs)]


class Config5Requests:
    """Poisson request stream over resident graphs: 45% increase, 45% decrease,
    2.5% add, 2.5% remove, 5% warm single-pair query, each on a uniformly
    chosen graph.  `arrivals(rate, count)` gives arrival times in seconds."""

    def __init__(self, adjs, seed: Optional[int] = None):
        ss = np.random.SeedSequence(seed_for(5) if seed is None else seed)
        _, _, r_seed = ss.spawn(3)
        self.rng = np.random.default_rng(r_seed)
        self.states = [GraphState(a, False) for a in adjs]

    def arrivals(self, rate: float, count: int) -> np.ndarray:
        return np.cumsum(self.rng.exponential(1.0 / rate, size=count))

    def next_request(self):
        g = int(self.rng.integers(0, len(self.states)))
        st = self.states[g]
        kinds = [k for k, _ in SERVE_MIX]
        probs = [p for _, p in SERVE_MIX]
        kind = kinds[int(self.rng.choice(len(kinds), p=probs))]
        if kind == REMOVE and len(st.live) <= 2:
            kind = DECREASE
        if kind == QUERY:
            i, j = self.rng.choice(len(st.live), size=2, replace=True)
            return g, kind, (st.live[int(i)], st.live[int(j)])
        return g, kind, make_update(self.rng, st, kind, wmin=1, wmax=10000, inc_max=20000)
