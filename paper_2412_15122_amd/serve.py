"""Serving many device-resident graphs with continuous batching.

A Server holds graphs (APSP matrices in HBM), admits them by HBM bytes, and
serves a stream of requests (edge updates, node additions and removals,
single-pair queries), each addressed to one graph and applied in that
graph's arrival order.

Scheduling (one host loop, polled):
  * arrivals go to their graph's FIFO queue;
  * a graph with queued requests that is not in HBM is admitted when its
    bytes fit the budget, after moving idle graphs (no queued or running
    work, least recently used first) out to host memory if needed;
  * schedule "lockstep" (default): whenever fewer than two batches are on
    the GPU, every resident graph's queued requests (up to a cap per graph)
    form the next batch, one lockstep launch in which all graphs' row sweeps
    share the whole GPU; requests that arrive while a batch runs join the
    next one, which is already queued behind it on the same stream, so the
    GPU never waits for the host; while the single calls keep up (at most
    small_batch queued and in flight, no batch in flight) requests run as
    single calls on that stream instead;
  * schedule "hybrid": edge updates and queries of idle graphs go to
    work-queue batches on free streams, node additions and removals to the
    single-update path on the graph's own stream, so launches for disjoint
    graphs overlap;
  * a request completes when the event recorded after its launch has fired;
    latency = completion time - arrival time.

serve_plain() runs the same requests without batching (one library call per
request, one stream) as the baseline.
"""
from __future__ import annotations

import collections
import dataclasses
import time
from typing import Dict, List, Optional, Sequence

import numpy as np

from . import _native as N
from .apsp import Graph, _torch
from .batch import Batch, QueryResult

LIGHT = ("increase", "decrease", "edge", "query")
HEAVY = ("add", "remove")


@dataclasses.dataclass
class Request:
    """kind: 'add' (args: w_out, w_in), 'remove' (id), 'increase' /
    'decrease' / 'edge' (u, v, w) or 'query' (i, j)."""
    graph: int
    kind: str
    args: tuple
    arrival: float = 0.0          # seconds from the start of the run
    done: Optional[float] = None  # seconds from the start of the run
    result: object = None         # add: new id; query: (dist, path ids)
    rid: int = -1

    @property
    def latency(self) -> Optional[float]:
        return None if self.done is None else self.done - self.arrival


class GraphSlot:
    def __init__(self, index: int, adj, undirected: bool, capacity: int, minimax: bool = False):
        self.index = index
        self.adj = adj
        self.undirected = undirected
        self.minimax = minimax
        self.capacity = capacity
        self.graph: Optional[Graph] = None
        self.queue: collections.deque = collections.deque()
        self.busy = False          # work in flight
        self.last_used = 0.0

    @property
    def resident(self) -> bool:
        return self.graph is not None and self.graph.resident


class Server:
    def __init__(self, graphs: Sequence, *, undirected: bool = False, budget_bytes: Optional[int] = None,
                 streams: int = 4, max_batch_items: int = 8192, batch_config: Optional[dict] = None,
                 headroom: int = 64, schedule: str = "lockstep", per_graph: int = 8, small_batch: int = 64,
                 minimax: bool = False):
        """graphs: adjacency matrices (numpy or torch, n x n int32).  Each is
        created in HBM (cold start) when first admitted.  budget_bytes:
        HBM the graphs may hold together (default 80% of free HBM).
        schedule: "lockstep" or "hybrid" (see the module notes); per_graph:
        requests of one graph a lockstep batch takes at most; small_batch:
        with no batch and fewer than this many single calls in flight, this
        many queued requests or fewer run as single calls instead (a
        lockstep launch has a fixed cost of a few grid barriers that one
        cheap update does not repay).  minimax: serve minimax (bottleneck)
        distances instead of shortest-path ones (a query's path is then a
        minimax path, found by the batch's candidate walk or by a single
        call's search, which may pick different ones)."""
        if schedule not in ("lockstep", "hybrid"):
            raise ValueError("schedule must be 'lockstep' or 'hybrid'")
        self.schedule = schedule
        self.per_graph = int(per_graph)
        self.small_batch = int(small_batch)
        if schedule == "lockstep":
            streams = 1
            batch_config = dict(batch_config or {"variant": 3, "use_graph": True})
        torch = _torch()
        self._torch = torch
        lib_bytes = N.load().apsp_required_bytes
        kind = 1 if undirected else 0
        self.slots: List[GraphSlot] = []
        for i, a in enumerate(graphs):
            n = int(a.shape[0])
            s = GraphSlot(i, a, undirected, n + headroom, minimax)
            s.nbytes = int(lib_bytes(s.capacity, kind))
            if s.nbytes == 0:
                raise ValueError(f"graph {i}: capacity {s.capacity} is out of range")
            self.slots.append(s)
        if budget_bytes is None:
            free, _ = torch.cuda.mem_get_info()
            budget_bytes = int(0.8 * free)
        self.budget = int(budget_bytes)
        big = max((s.nbytes for s in self.slots), default=0)
        if big > self.budget:
            raise ValueError("the largest graph does not fit the HBM budget")
        self.used = 0
        self.streams = [torch.cuda.Stream() for _ in range(max(1, streams))]
        cfg = dict(batch_config or {})
        self.batches = [Batch(len(self.slots), max_batch_items, **cfg) for _ in self.streams]
        self.max_batch_items = int(max_batch_items)
        self.stream_busy = [None] * len(self.streams)   # (event, requests, slots) per stream
        self.heavy_inflight: List[tuple] = []           # (event, request, slot)
        self.lock_inflight: collections.deque = collections.deque()  # lockstep: (event, requests, slots, results, batch)
        self.lock_depth = 2 if schedule == "lockstep" else 0
        if schedule == "lockstep":
            self.batches.append(Batch(len(self.slots), max_batch_items, **cfg))
        self.stats = collections.Counter()
        self.n_done = 0

    # -- admission ------------------------------------------------------------
    def _admit(self, s: GraphSlot, now: float) -> bool:
        if s.resident:
            return True
        if self.used + s.nbytes > self.budget:
            # idle graphs first (least recently used first), then graphs with
            # no work in flight whose oldest queued request is newer than
            # this graph's, so that a graph under steady traffic cannot keep
            # its HBM while an older request waits
            head = s.queue[0].arrival if s.queue else float("inf")
            idle = sorted((x for x in self.slots if x.resident and not x.busy
                           and (not x.queue or x.queue[0].arrival > head)),
                          key=lambda x: (bool(x.queue), x.last_used))
            for x in idle:
                if self.used + s.nbytes <= self.budget:
                    break
                x.graph.swap_out()
                self.used -= x.nbytes
                self.stats["evictions"] += 1
            if self.used + s.nbytes > self.budget:
                return False
        stream = self.streams[s.index % len(self.streams)]
        with self._torch.cuda.stream(stream):
            if s.graph is None:
                s.graph = Graph(s.adj, undirected=s.undirected, capacity=s.capacity, minimax=s.minimax)
                self.stats["cold_starts"] += 1
            else:
                s.graph.swap_in()
                self.stats["swap_ins"] += 1
        s.graph.set_stream(stream)
        self.used += s.nbytes
        s.last_used = now
        return True

    # -- dispatch ---------------------------------------------------------------
    def _run_heavy(self, s: GraphSlot, r: Request):
        g = s.graph
        torch = self._torch
        # spreading heavy requests over the streams lets them overlap;
        # set_stream orders the graph's earlier work (a cold start) first
        self._rr = (getattr(self, "_rr", -1) + 1) % len(self.streams)
        g.set_stream(self.streams[self._rr])
        with torch.cuda.stream(g._stream):
            if r.kind == "add":
                r.result = g.add_node(r.args[0], None if g.undirected else r.args[1])
            else:
                g.remove_node(r.args[0])
            ev = torch.cuda.Event()
            ev.record(g._stream)
        self.heavy_inflight.append((ev, r, s))
        s.busy = True
        self.stats["heavy"] += 1

    def _launch_batch(self, si: int, work: List[tuple]):
        """work: (slot, [requests]) with light requests only."""
        torch = self._torch
        stream = self.streams[si]
        graphs = [s.graph for s, _ in work]
        items, reqs = [], []
        for gi, (s, rs) in enumerate(work):
            # idle graphs join the batch's stream: no cross-stream waits
            s.graph.set_stream(stream)
            for r in rs:
                if r.kind == "query":
                    items.append(("query", gi, r.args[0], r.args[1]))
                else:
                    items.append(("edge", gi, r.args[0], r.args[1], r.args[2]))
                reqs.append(r)
            s.busy = True
        with torch.cuda.stream(stream):
            res = self.batches[si].run(graphs, items, stream=stream)
            ev = torch.cuda.Event()
            ev.record(stream)
        self.stream_busy[si] = (ev, reqs, [s for s, _ in work], res)
        self.stats["batches"] += 1
        self.stats["batched_items"] += len(items)

    def _complete(self, now: float):
        while self.lock_inflight and self.lock_inflight[0][0].query():
            _, reqs, slots, res, _bi = self.lock_inflight.popleft()
            for r, x in zip(reqs, res):
                if r.kind == "query":
                    r.result = x.get() if isinstance(x, QueryResult) else x
                elif r.kind == "add":
                    r.result = x
                r.done = now
                self.n_done += 1
            for s in slots:
                s.inflight -= 1
                s.busy = s.inflight > 0
                s.last_used = now
        for si, ent in enumerate(self.stream_busy):
            if ent is None or not ent[0].query():
                continue
            _, reqs, slots, res = ent
            for r, x in zip(reqs, res):
                if r.kind == "query":
                    r.result = x.get()
                r.done = now
                self.n_done += 1
            for s in slots:
                s.busy = False
                s.last_used = now
            self.stream_busy[si] = None
        keep = []
        for ev, r, s in self.heavy_inflight:
            if ev.query():
                r.done = now
                self.n_done += 1
                s.busy = False
                s.last_used = now
            else:
                keep.append((ev, r, s))
        self.heavy_inflight = keep

    def _launch_lockstep(self):
        """Every resident graph's queued requests (up to per_graph each) as
        one lockstep batch behind the ones already on the stream, or, at
        light load, as single calls."""
        torch = self._torch
        work, n_items = [], 0
        # a graph waiting for admission holds back graphs whose queue is
        # newer, so they drain and one of them can make room
        waiting = [s.queue[0].arrival for s in self.slots if s.queue and not s.resident]
        oldest_wait = min(waiting) if waiting else float("inf")
        ready = sorted((s for s in self.slots if s.queue and s.resident and s.queue[0].arrival <= oldest_wait),
                       key=lambda s: s.queue[0].arrival)
        if not ready:
            return
        # light load: a few requests go out as single calls while no batch is
        # in flight and few single calls are; a longer queue (the single
        # calls fall behind) goes out as a lockstep batch
        n_batches = sum(1 for e in self.lock_inflight if e[4] is not None)
        n_single = len(self.lock_inflight) - n_batches
        queued = sum(min(len(s.queue), self.per_graph) for s in ready)
        if queued <= self.small_batch and n_batches == 0:
            if n_single < self.small_batch:
                self._run_single([(s, [s.queue.popleft() for _ in range(min(len(s.queue), self.per_graph))])
                                  for s in ready])
            return
        if n_batches >= self.lock_depth:
            return
        for s in ready:
            take = []
            while s.queue and len(take) < self.per_graph and n_items + len(take) < self.max_batch_items:
                take.append(s.queue.popleft())
            if take:
                work.append((s, take))
                n_items += len(take)
        graphs = [s.graph for s, _ in work]
        items, reqs = [], []
        for gi, (s, rs) in enumerate(work):
            for r in rs:
                if r.kind == "query":
                    items.append(("query", gi, r.args[0], r.args[1]))
                elif r.kind == "add":
                    items.append(("add", gi, r.args[0], r.args[1]))
                elif r.kind == "remove":
                    items.append(("remove", gi, r.args[0]))
                else:
                    items.append(("edge", gi, r.args[0], r.args[1], r.args[2]))
                reqs.append(r)
            s.inflight = getattr(s, "inflight", 0) + 1
            s.busy = True
        bi = self._next_batch = (getattr(self, "_next_batch", -1) + 1) % len(self.batches)
        stream = self.streams[0]
        with torch.cuda.stream(stream):
            res = self.batches[bi].run(graphs, items, stream=stream)
            ev = torch.cuda.Event()
            ev.record(stream)
        self.lock_inflight.append((ev, reqs, [s for s, _ in work], res, bi))
        self.stats["batches"] += 1
        self.stats["batched_items"] += len(items)

    def _run_single(self, work: List[tuple]):
        """A few requests, one library call each on the batch stream (a
        query waits for its answer), each completed by its own event."""
        torch = self._torch
        stream = self.streams[0]
        with torch.cuda.stream(stream):
            for s, rs in work:
                g = s.graph
                for r in rs:
                    if r.kind == "add":
                        x = g.add_node(r.args[0], None if g.undirected else r.args[1])
                    elif r.kind == "remove":
                        x = g.remove_node(r.args[0])
                    elif r.kind == "query":
                        x = g.query(r.args[0], r.args[1])
                    else:
                        x = g.update_edge(r.args[0], r.args[1], r.args[2])
                    ev = torch.cuda.Event()
                    ev.record(stream)
                    s.inflight = getattr(s, "inflight", 0) + 1
                    s.busy = True
                    self.lock_inflight.append((ev, [r], [s], [x], None))
                    self.stats["single"] += 1

    def _dispatch(self, now: float):
        # admission, oldest head request first
        waiting = sorted((s for s in self.slots if s.queue and not s.resident), key=lambda s: s.queue[0].arrival)
        for s in waiting:
            self._admit(s, now)
        if self.schedule == "lockstep":
            self._launch_lockstep()
            return
        free = [i for i, e in enumerate(self.stream_busy) if e is None]
        work, n_items = [], 0
        for s in sorted((s for s in self.slots if s.queue and s.resident and not s.busy),
                        key=lambda s: s.queue[0].arrival):
            head = s.queue[0]
            if head.kind in HEAVY:
                self._run_heavy(s, s.queue.popleft())
                continue
            if not free:
                continue
            take = []
            while s.queue and s.queue[0].kind in LIGHT and n_items + len(take) < self.max_batch_items:
                take.append(s.queue.popleft())
            if take:
                work.append((s, take))
                n_items += len(take)
        if work:
            self._launch_batch(free[0], work)

    # -- the loop -----------------------------------------------------------------
    def run(self, requests: Sequence[Request]) -> Dict[str, float]:
        """Serve `requests` in real time (arrival times in seconds from the
        start); returns summary statistics.  Every request's `done` and
        `result` are filled in."""
        torch = self._torch
        for i, r in enumerate(requests):
            if r.rid < 0:
                r.rid = i
            r.done = None
        pending = collections.deque(sorted(requests, key=lambda r: r.arrival))
        torch.cuda.synchronize()
        self.n_done = 0
        t0 = time.perf_counter()
        while self.n_done < len(requests):
            now = time.perf_counter() - t0
            while pending and pending[0].arrival <= now:
                r = pending.popleft()
                self.slots[r.graph].queue.append(r)
            self._complete(now)
            self._dispatch(now)
        wall = time.perf_counter() - t0
        return summarize(requests, wall)

    def preload(self) -> int:
        """Admit graphs in index order while they fit (cold starts before a
        timed run); returns how many are resident."""
        for s in self.slots:
            if self.used + s.nbytes <= self.budget:
                self._admit(s, 0.0)
        self._torch.cuda.synchronize()
        return sum(1 for s in self.slots if s.resident)

    def graph(self, i: int) -> Graph:
        s = self.slots[i]
        if s.graph is not None and not s.resident:
            self._admit(s, 0.0)
        return s.graph

    def close(self):
        for b in self.batches:
            b.close()
        for s in self.slots:
            if s.graph is not None:
                s.graph.close()


def summarize(requests: Sequence[Request], wall: float) -> Dict[str, float]:
    lat = np.array([r.latency for r in requests if r.latency is not None])
    upd = sum(1 for r in requests if r.kind != "query")
    return {
        "requests": len(requests),
        "updates": upd,
        "wall_s": wall,
        "updates_per_s": upd / wall if wall > 0 else 0.0,
        "requests_per_s": len(requests) / wall if wall > 0 else 0.0,
        "p50_ms": float(np.percentile(lat, 50) * 1e3) if lat.size else None,
        "p99_ms": float(np.percentile(lat, 99) * 1e3) if lat.size else None,
        "mean_ms": float(lat.mean() * 1e3) if lat.size else None,
    }


def serve_plain(graphs: Sequence[Graph], requests: Sequence[Request]) -> Dict[str, float]:
    """Baseline: the same requests in arrival order, one library call each,
    on the current stream, no batching; a request completes when the event
    after its call fires."""
    torch = _torch()
    pending = collections.deque(sorted(requests, key=lambda r: r.arrival))
    inflight = collections.deque()
    stream = torch.cuda.current_stream()
    for g in graphs:
        g.set_stream(stream)
    for r in requests:
        r.done = None
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    n_done = 0
    while n_done < len(requests):
        now = time.perf_counter() - t0
        while pending and pending[0].arrival <= now:
            r = pending.popleft()
            g = graphs[r.graph]
            if r.kind == "add":
                r.result = g.add_node(r.args[0], None if g.undirected else r.args[1])
            elif r.kind == "remove":
                g.remove_node(r.args[0])
            elif r.kind == "query":
                r.result = g.query(r.args[0], r.args[1])   # synchronous
            else:
                g.update_edge(r.args[0], r.args[1], r.args[2])
            ev = torch.cuda.Event()
            ev.record(stream)
            inflight.append((ev, r))
        now = time.perf_counter() - t0
        while inflight and inflight[0][0].query():
            inflight.popleft()[1].done = now
            n_done += 1
    wall = time.perf_counter() - t0
    return summarize(requests, wall)


def requests_from_stream(gen, rate: float, count: int) -> List[Request]:
    """Draw `count` requests from a Config5Requests-style generator with
    Poisson arrivals at `rate` per second."""
    arr = gen.arrivals(rate, count)
    out = []
    for t in range(count):
        g, kind, payload = gen.next_request()
        if kind == "query":
            r = Request(g, "query", tuple(int(x) for x in payload), float(arr[t]))
        elif kind == "add":
            r = Request(g, "add", (payload.w_out, payload.w_in), float(arr[t]))
        elif kind == "remove":
            r = Request(g, "remove", (payload.u,), float(arr[t]))
        else:
            r = Request(g, kind, (payload.u, payload.v, payload.w), float(arr[t]))
        r.rid = t
        out.append(r)
    return out
