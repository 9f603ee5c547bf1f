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
  * every resident graph with nothing in flight contributes work: the
    longest run of light requests at the head of its queue (edge updates and
    queries) joins the next batched launch (one persistent launch over all
    such graphs, on a free stream), while a heavy request at the head (node
    addition or removal, whose O(n^2) sweeps need the whole GPU) runs through
    the single-update path on the graph's own stream;
  * launches are asynchronous: requests that arrive while earlier work is on
    the GPU are taken by the next launch as soon as their graph is free, and
    launches for disjoint graphs overlap on different streams;
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
from .batch import Batch

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
    def __init__(self, index: int, adj, undirected: bool, capacity: int):
        self.index = index
        self.adj = adj
        self.undirected = undirected
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
                 headroom: int = 64):
        """graphs: adjacency matrices (numpy or torch, n x n int32).  Each is
        created in HBM (cold start) when first admitted.  budget_bytes:
        HBM the graphs may hold together (default 80% of free HBM)."""
        torch = _torch()
        self._torch = torch
        lib_bytes = N.load().apsp_required_bytes
        kind = 1 if undirected else 0
        self.slots: List[GraphSlot] = []
        for i, a in enumerate(graphs):
            n = int(a.shape[0])
            s = GraphSlot(i, a, undirected, n + headroom)
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
        self.stats = collections.Counter()
        self.n_done = 0

    # -- admission ------------------------------------------------------------
    def _admit(self, s: GraphSlot, now: float) -> bool:
        if s.resident:
            return True
        if self.used + s.nbytes > self.budget:
            idle = sorted((x for x in self.slots if x.resident and not x.busy and not x.queue),
                          key=lambda x: x.last_used)
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
                s.graph = Graph(s.adj, undirected=s.undirected, capacity=s.capacity)
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
        # the graph is idle (its earlier work has completed), so it may move
        # to any stream; spreading heavy requests lets them overlap
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

    def _dispatch(self, now: float):
        # admission, oldest head request first
        waiting = sorted((s for s in self.slots if s.queue and not s.resident), key=lambda s: s.queue[0].arrival)
        for s in waiting:
            self._admit(s, now)
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
