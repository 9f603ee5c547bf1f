"""Batched updates over many device-resident graphs (apsp_batch_* in the C ABI).

A Batch owns a device workspace and runs, in one persistent launch, any
number of graphs' queued updates and queries; each graph's items are applied
in the order given, with the same results as the single calls on Graph.

Items are tuples:
    ("add", graph_index, w_out, w_in)    w_in is ignored for undirected graphs
    ("remove", graph_index, node_id)
    ("edge", graph_index, u, v, w)
    ("query", graph_index, i, j)
Weights are numpy arrays or CUDA tensors (one entry per live node, ascending
ids at that point of the graph's queue).
"""
from __future__ import annotations

import ctypes
import sys
from typing import List, Optional, Sequence

import numpy as np

from . import _native as N
from .apsp import Graph, _device_int32, _torch

_OPS = {"add": N.APSP_OP_ADD_NODE, "remove": N.APSP_OP_REMOVE_NODE, "edge": N.APSP_OP_UPDATE_EDGE,
        "query": N.APSP_OP_QUERY}


class QueryResult:
    """A batched query's answer; read it after the stream has run the batch."""

    def __init__(self, buf, offset: int, cap: int):
        self._buf = buf
        self._off = offset
        self._cap = cap

    def get(self):
        """(distance, path ids); waits for the device."""
        v = self._buf[self._off:self._off + self._cap].cpu().numpy()
        if v[2] != 0:
            raise RuntimeError("no shortest path found on the device")
        return int(v[0]), [int(x) for x in v[3:3 + v[1]]]


class Batch:
    def __init__(self, max_graphs: int, max_items: int, *, grid: int = 0, order: int = 0, variant: int = 0,
                 use_graph: bool = True):
        torch = _torch()
        self._lib = N.load()
        nbytes = int(self._lib.apsp_batch_workspace_bytes(int(max_graphs), int(max_items)))
        if nbytes == 0:
            raise ValueError("max_graphs and max_items must be >= 1")
        self._ws = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
        ptr = (self._ws.data_ptr() + 255) & ~255
        h = ctypes.c_void_p()
        N.check(self._lib.apsp_batch_create(ptr, nbytes, int(max_graphs), int(max_items), ctypes.byref(h)),
                "apsp_batch_create")
        self._h = h
        self.max_graphs = int(max_graphs)
        self.max_items = int(max_items)
        self.set_config(grid=grid, order=order, variant=variant, use_graph=use_graph)

    def set_config(self, *, grid: int = 0, order: int = 0, variant: int = 0, use_graph: bool = True) -> None:
        N.check(self._lib.apsp_batch_set_config(self._h, int(grid), int(order), int(variant), int(bool(use_graph))),
                "apsp_batch_set_config")
        self.config = {"grid": int(grid), "order": int(order), "variant": int(variant), "use_graph": bool(use_graph)}

    def close(self) -> None:
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.apsp_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        # at interpreter exit the HIP runtime may already be torn down: make
        # no HIP call then (the process releases everything anyway)
        if sys.is_finalizing():
            return
        try:
            self.close()
        except Exception:
            pass

    def run(self, graphs: Sequence[Graph], items: Sequence[tuple], *, stream=None) -> List[object]:
        """Enqueue the batch; returns, per item, the new id (add), a
        QueryResult (query) or None."""
        return self.submit(self.prepare(graphs, items), stream=stream)

    def prepare(self, graphs: Sequence[Graph], items: Sequence[tuple]) -> "Prepared":
        """Marshal the items (device weight vectors, query outputs) once;
        the result can be submitted to graphs in the state it was made for."""
        torch = _torch()
        ng = len(graphs)
        arr = (N.BatchItem * max(len(items), 1))()
        keep = []
        results: List[object] = [None] * len(items)
        # live counts along each graph's queue, to size weight checks and query outputs
        live = [g.num_nodes() for g in graphs]
        qcaps = []
        for t, it in enumerate(items):
            op = it[0]
            gi = int(it[1])
            if not 0 <= gi < ng:
                raise ValueError(f"item {t}: graph index out of range")
            x = arr[t]
            x.graph = gi
            x.op = _OPS[op]
            if op == "add":
                n = live[gi]
                if n:
                    wo = _device_int32(it[2]).reshape(-1)
                    if wo.numel() != n:
                        raise ValueError(f"item {t}: w_out needs {n} entries")
                    keep.append(wo)
                    x.w_out_dev = wo.data_ptr()
                    if not graphs[gi].undirected:
                        if len(it) < 4 or it[3] is None:
                            raise ValueError(f"item {t}: w_in is required for a directed graph")
                        wi = _device_int32(it[3]).reshape(-1)
                        if wi.numel() != n:
                            raise ValueError(f"item {t}: w_in needs {n} entries")
                        keep.append(wi)
                        x.w_in_dev = wi.data_ptr()
                live[gi] += 1
            elif op == "remove":
                x.u = int(it[2])
                live[gi] -= 1
            elif op == "edge":
                x.u, x.v, x.w = int(it[2]), int(it[3]), int(it[4])
            elif op == "query":
                x.u, x.v = int(it[2]), int(it[3])
                qcaps.append((t, 3 + live[gi]))
            else:
                raise ValueError(f"item {t}: unknown op {op!r}")
        if qcaps:
            total = sum(c for _, c in qcaps)
            qbuf = torch.empty(total, dtype=torch.int32, device="cuda")
            off = 0
            for t, c in qcaps:
                arr[t].out_dev = qbuf.data_ptr() + 4 * off
                arr[t].out_cap = c
                results[t] = QueryResult(qbuf, off, c)
                off += c
            keep.append(qbuf)
        return Prepared(graphs, items, arr, keep, results)

    def submit(self, prep: "Prepared", *, graphs: Optional[Sequence[Graph]] = None, stream=None) -> List[object]:
        """Run a prepared batch (on `graphs`, default the ones it was made
        for: e.g. clones in the same state)."""
        torch = _torch()
        stream = stream or torch.cuda.current_stream()
        graphs = prep.graphs if graphs is None else graphs
        ng = len(graphs)
        hs = (ctypes.c_void_p * max(ng, 1))(*[g._h.value for g in graphs])
        ids = (ctypes.c_int32 * max(len(prep.items), 1))()
        N.check(self._lib.apsp_batch_run(self._h, hs, ng, prep.arr, len(prep.items), stream.cuda_stream, ids),
                "apsp_batch_run")
        results = list(prep.results)
        for t, it in enumerate(prep.items):
            if it[0] == "add":
                results[t] = int(ids[t])
        for t in prep.keep:
            t.record_stream(stream)
        self._keep = prep.keep  # weight vectors stay referenced until the next run
        return results


    def status(self) -> None:
        """Wait for the last run; raises if a lockstep barrier timed out."""
        N.check(self._lib.apsp_batch_status(self._h), "apsp_batch_status")

    def phase_times(self):
        """Lockstep diagnostics of the last run: microseconds at the end of
        each step's phases (see apsp_batch_phase_times)."""
        buf = (ctypes.c_double * 96)()
        cnt = ctypes.c_int32()
        N.check(self._lib.apsp_batch_phase_times(self._h, buf, 96, ctypes.byref(cnt)), "apsp_batch_phase_times")
        return np.array(buf[:cnt.value])

    def graph_times(self, num_graphs: int):
        """(start_us, end_us) per graph of the last run (waits for it)."""
        a = (ctypes.c_double * max(num_graphs, 1))()
        b = (ctypes.c_double * max(num_graphs, 1))()
        N.check(self._lib.apsp_batch_graph_times(self._h, a, b, int(num_graphs)), "apsp_batch_graph_times")
        return np.array(a[:num_graphs]), np.array(b[:num_graphs])


class Prepared:
    def __init__(self, graphs, items, arr, keep, results):
        self.graphs = list(graphs)
        self.items = list(items)
        self.arr = arr
        self.keep = keep
        self.results = results
