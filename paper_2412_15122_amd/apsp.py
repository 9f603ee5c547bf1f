"""Python face of the HIP library: a device-resident graph with its APSP matrix.

Every method marshals arguments and calls the C ABI (include/apsp.h); all
arithmetic runs in the library's gfx950 kernels.  torch supplies the device
buffer and the stream only.
"""
from __future__ import annotations

import ctypes
import sys
from typing import List, Optional, Sequence, Tuple

import numpy as np

from . import _native as N

INF = N.APSP_INF


def _torch():
    import torch
    return torch


def _device_int32(x):
    """A contiguous int32 CUDA tensor holding x (numpy, list or tensor)."""
    torch = _torch()
    if isinstance(x, torch.Tensor):
        t = x
    else:
        t = torch.from_numpy(np.ascontiguousarray(np.asarray(x, dtype=np.int32)))
    return t.to(device="cuda", dtype=torch.int32).contiguous()


def _path_bits(minimax: bool, widest: bool) -> int:
    """The kind bits of a graph's path problem."""
    return N.APSP_WIDEST if widest else (N.APSP_MINIMAX if minimax else 0)


class Graph:
    """A dense weighted graph whose APSP matrix lives on the GPU.

    Graph(adj, undirected=False, capacity=None, minimax=False) runs the cold
    start (apsp_cold).  `adj` is an n x n int32 matrix (numpy or torch),
    absent edges APSP_INF, diagonal ignored.  Ids are 0..n-1; added nodes
    get max_id + 1.  minimax=True keeps minimax (bottleneck) distances
    instead of shortest-path ones (APSP_MINIMAX); widest=True keeps widest
    (maximum-capacity) paths: `adj` then holds capacities in
    [0, APSP_INF - 1] (APSP_INF: no edge), and every matrix, distance and
    weight read back is a width (APSP_WIDEST).
    """

    def __init__(self, adj, *, undirected: bool = False, capacity: Optional[int] = None, minimax: bool = False,
                 widest: bool = False):
        torch = _torch()
        self._lib = N.load()
        A = _device_int32(adj)
        if A.dim() != 2 or A.shape[0] != A.shape[1]:
            raise ValueError("adjacency must be square")
        n = int(A.shape[0])
        cap = int(capacity if capacity is not None else max(n, 1))
        self.kind = N.APSP_UNDIRECTED if undirected else N.APSP_DIRECTED
        self.undirected = bool(undirected)
        self.widest = bool(widest)
        self.minimax = bool(minimax) or self.widest
        nbytes = int(self._lib.apsp_required_bytes(cap, self.kind))
        if nbytes == 0:
            raise ValueError(f"invalid capacity {cap}")
        self._buf = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
        base = self._buf.data_ptr()
        self._ptr = (base + 255) & ~255
        self._nbytes = nbytes
        self.capacity = cap
        self._stream = torch.cuda.current_stream()
        h = ctypes.c_void_p()
        kind = self.kind | _path_bits(self.minimax, self.widest)
        st = self._lib.apsp_cold(A.data_ptr() if n else None, n, A.stride(0) if n else 0, kind, cap,
                                 self._ptr, nbytes, self._stream.cuda_stream, ctypes.byref(h))
        N.check(st, "apsp_cold")
        self._h = h
        self._keep = []

    @classmethod
    def from_matrix(cls, adj, dist, *, undirected: bool = False, capacity: Optional[int] = None,
                    minimax: bool = False, ids: Optional[Sequence[int]] = None, next_id: Optional[int] = None,
                    exact: bool = False, widest: bool = False) -> "Graph":
        """A graph whose distance matrix is already known (apsp_import): the
        paper's starting point, where the old matrix is given and only the
        updates are paid for.  `dist` is n x n in the order of `adj`'s rows;
        `ids` (ascending) name those rows (default 0..n-1); `next_id` is the
        id the next add_node returns (default: the largest id + 1).  exact=True also
        recomputes cold and compares; otherwise only the O(n^2) checks of a
        distance matrix are made.  Raises ApspError if a check fails."""
        torch = _torch()
        lib = N.load()
        A = _device_int32(adj)
        Dm = _device_int32(dist)
        if A.dim() != 2 or A.shape[0] != A.shape[1] or tuple(Dm.shape) != tuple(A.shape):
            raise ValueError("adjacency and distance matrix must be square and of one size")
        n = int(A.shape[0])
        if ids is not None and len(ids) != n:
            raise ValueError(f"ids must have {n} entries")
        cap = int(capacity if capacity is not None else max(n, 1))
        kind = N.APSP_UNDIRECTED if undirected else N.APSP_DIRECTED
        nbytes = int(lib.apsp_required_bytes(cap, kind))
        if nbytes == 0:
            raise ValueError(f"invalid capacity {cap}")
        buf = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
        ptr = (buf.data_ptr() + 255) & ~255
        stream = torch.cuda.current_stream()
        id_arr = None
        if ids is not None and n:
            id_arr = (ctypes.c_int32 * n)(*[int(x) for x in ids])
        h = ctypes.c_void_p()
        st = lib.apsp_import(A.data_ptr() if n else None, A.stride(0) if n else 0,
                             Dm.data_ptr() if n else None, Dm.stride(0) if n else 0, n, id_arr,
                             -1 if next_id is None else int(next_id),
                             kind | _path_bits(minimax, widest), cap, ptr, nbytes, stream.cuda_stream,
                             N.APSP_IMPORT_EXACT if exact else N.APSP_IMPORT_TRUSTED, ctypes.byref(h))
        N.check(st, "apsp_import")
        return cls._from_handle(lib, h, buf, ptr, nbytes, cap, kind, stream, bool(minimax) or bool(widest),
                                bool(widest))

    def grow(self, capacity: int) -> "Graph":
        """A copy of this graph with `capacity` node slots (apsp_grow): every
        used slot keeps its place, ids, distances and weights, so the copy
        behaves as this graph would with more room.  O(n^2) device copies;
        this graph is left unchanged."""
        torch = _torch()
        nbytes = int(self._lib.apsp_required_bytes(int(capacity), self.kind))
        if nbytes == 0:
            raise ValueError(f"invalid capacity {capacity}")
        buf = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
        ptr = (buf.data_ptr() + 255) & ~255
        stream = torch.cuda.current_stream()
        h = ctypes.c_void_p()
        N.check(self._lib.apsp_grow(self._h, int(capacity), ptr, nbytes, stream.cuda_stream, ctypes.byref(h)),
                "apsp_grow")
        return Graph._from_handle(self._lib, h, buf, ptr, nbytes, int(capacity), self.kind, stream, self.minimax,
                                  self.widest)

    @classmethod
    def _from_handle(cls, lib, h, buf, ptr, nbytes, cap, kind, stream, minimax=False, widest=False):
        g = cls.__new__(cls)
        g._lib = lib
        g._h = h
        g._buf = buf
        g._ptr = ptr
        g._nbytes = nbytes
        g.capacity = cap
        g.kind = kind
        g.undirected = kind == N.APSP_UNDIRECTED
        g.minimax = minimax
        g.widest = widest
        g._stream = stream
        g._keep = []
        return g

    def clone(self) -> "Graph":
        """An independent copy of this graph (apsp_graph_clone)."""
        torch = _torch()
        buf = torch.empty(self._nbytes + 256, dtype=torch.uint8, device="cuda")
        ptr = (buf.data_ptr() + 255) & ~255
        stream = torch.cuda.current_stream()
        if stream.cuda_stream != self._stream.cuda_stream:
            stream.wait_stream(self._stream)  # the source's queued updates come first
        h = ctypes.c_void_p()
        N.check(self._lib.apsp_graph_clone(self._h, ptr, self._nbytes, stream.cuda_stream, ctypes.byref(h)),
                "apsp_graph_clone")
        if stream.cuda_stream != self._stream.cuda_stream:
            self._stream.wait_stream(stream)  # and the source's later updates after the copy
        return Graph._from_handle(self._lib, h, buf, ptr, self._nbytes, self.capacity, self.kind, stream,
                                  self.minimax, self.widest)

    @property
    def nbytes(self) -> int:
        """Device bytes the graph holds (apsp_required_bytes)."""
        return self._nbytes

    @property
    def resident(self) -> bool:
        return self._buf is not None and self._buf.is_cuda

    def swap_out(self) -> None:
        """Copy the graph's device buffer to host memory and release the HBM
        (the handle keeps the ids and bookkeeping)."""
        torch = _torch()
        if not self.resident:
            return
        off = self._ptr - self._buf.data_ptr()
        host = torch.empty(self._nbytes, dtype=torch.uint8, pin_memory=True)
        with torch.cuda.stream(self._stream):
            host.copy_(self._buf[off:off + self._nbytes], non_blocking=True)
        self._stream.synchronize()
        # from here on the library refuses every call that would touch the
        # old buffer, until swap_in relocates the graph
        N.check(self._lib.apsp_graph_detach(self._h), "apsp_graph_detach")
        self._buf = host
        self._ptr = None

    def swap_in(self) -> None:
        """Bring a swapped-out graph back into HBM (apsp_graph_relocate)."""
        torch = _torch()
        if self.resident:
            return
        buf = torch.empty(self._nbytes + 256, dtype=torch.uint8, device="cuda")
        ptr = (buf.data_ptr() + 255) & ~255
        off = ptr - buf.data_ptr()
        with torch.cuda.stream(self._stream):
            buf[off:off + self._nbytes].copy_(self._buf, non_blocking=True)
        N.check(self._lib.apsp_graph_relocate(self._h, ptr, self._nbytes), "apsp_graph_relocate")
        self._stream.synchronize()
        self._buf = buf
        self._ptr = ptr

    def set_stream(self, stream) -> None:
        """Issue the graph's later work on `stream`; work already queued on
        the old stream (a cold start, an update) is ordered before it by an
        event, without waiting on the host."""
        old = getattr(self, "_stream", None)
        if old is not None and old.cuda_stream != stream.cuda_stream:
            ev = _torch().cuda.Event()
            ev.record(old)
            stream.wait_event(ev)
        N.check(self._lib.apsp_set_stream(self._h, stream.cuda_stream), "apsp_set_stream")
        self._stream = stream

    # -- lifetime ------------------------------------------------------------
    def close(self) -> None:
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.apsp_graph_destroy(self._h)
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

    # -- updates --------------------------------------------------------------
    def _join(self):
        """The current stream, after making the graph's stream wait for it
        (work the caller queued there, e.g. a tensor it filled, comes first)."""
        cur = _torch().cuda.current_stream()
        if cur.cuda_stream != self._stream.cuda_stream:
            self._stream.wait_stream(cur)
        return cur

    def add_node(self, w_out, w_in=None) -> int:
        """Add a node; w_out[t] / w_in[t] are the weights to / from the t-th
        live node in ascending-id order.  Returns the new id."""
        torch = _torch()
        n = self.num_nodes()
        if n and not self.undirected and w_in is None:
            raise ValueError("w_in is required for a directed graph")
        self._join()
        with torch.cuda.stream(self._stream):
            wo = _device_int32(w_out).reshape(-1) if n else None
            wi = _device_int32(w_in).reshape(-1) if n and not self.undirected else None
            if n and (wo.numel() != n or (wi is not None and wi.numel() != n)):
                raise ValueError(f"weight vectors must have {n} entries")
            nid = self.add_node_device(wo.data_ptr() if n else None, wi.data_ptr() if wi is not None else None)
            for t in (wo, wi):
                if t is not None:
                    t.record_stream(self._stream)  # not reused before the kernels have read it
        return nid

    def add_node_device(self, w_out_ptr, w_in_ptr) -> int:
        """add_node with device pointers (length = live count)."""
        nid = ctypes.c_int32()
        N.check(self._lib.apsp_add_node(self._h, w_out_ptr, w_in_ptr, ctypes.byref(nid)), "apsp_add_node")
        return int(nid.value)

    def remove_node(self, node_id: int) -> None:
        N.check(self._lib.apsp_remove_node(self._h, int(node_id)), "apsp_remove_node")

    def update_edge(self, u: int, v: int, w: int) -> None:
        N.check(self._lib.apsp_update_edge(self._h, int(u), int(v), int(w)), "apsp_update_edge")

    def update_edge_noalloc(self, u: int, v: int, w: int) -> None:
        """update_edge with the library's static working memory (no device
        allocation; capacity <= APSP_NOALLOC_MAX_CAPACITY)."""
        N.check(self._lib.apsp_update_edge_noalloc(self._h, int(u), int(v), int(w)), "apsp_update_edge_noalloc")

    def recompute_cold(self) -> None:
        N.check(self._lib.apsp_recompute_cold(self._h), "apsp_recompute_cold")

    # -- reads ------------------------------------------------------------------
    def num_nodes(self) -> int:
        n = ctypes.c_int32()
        N.check(self._lib.apsp_node_count(self._h, ctypes.byref(n)), "apsp_node_count")
        return int(n.value)

    def next_id(self) -> int:
        """The id the next add_node returns (ids are never reused)."""
        x = ctypes.c_int32()
        N.check(self._lib.apsp_next_id(self._h, ctypes.byref(x)), "apsp_next_id")
        return int(x.value)

    def ids(self) -> List[int]:
        n = self.num_nodes()
        buf = (ctypes.c_int32 * max(n, 1))()
        cnt = ctypes.c_int32()
        N.check(self._lib.apsp_node_ids(self._h, buf, n, ctypes.byref(cnt)), "apsp_node_ids")
        return list(buf[: cnt.value])

    def matrix_device(self, which: str = "D"):
        """D (or A) in ascending-id order as a new device tensor, ready for
        use on the current stream."""
        torch = _torch()
        n = self.num_nodes()
        out = torch.empty((n, n), dtype=torch.int32, device="cuda")
        cur = self._join()
        fn = self._lib.apsp_read_matrix if which == "D" else self._lib.apsp_read_adjacency
        N.check(fn(self._h, out.data_ptr() if n else None, max(n, 1)), "apsp_read")
        if cur.cuda_stream != self._stream.cuda_stream:
            cur.wait_stream(self._stream)
            out.record_stream(self._stream)
        return out

    def matrix(self) -> np.ndarray:
        """Distance matrix in ascending-id order (host copy)."""
        return self.matrix_device("D").cpu().numpy()

    def adjacency(self) -> np.ndarray:
        return self.matrix_device("A").cpu().numpy()

    def query(self, i: int, j: int) -> Tuple[int, List[int]]:
        """(distance, shortest path as ids) from i to j."""
        cap = self.num_nodes()
        buf = (ctypes.c_int32 * max(cap, 1))()
        dist = ctypes.c_int32()
        ln = ctypes.c_int32()
        N.check(self._lib.apsp_query(self._h, int(i), int(j), ctypes.byref(dist), buf, cap, ctypes.byref(ln)),
                "apsp_query")
        return int(dist.value), list(buf[: ln.value])

    def query_nodes(self, i: int, j: int) -> Tuple[int, List[int], List[int]]:
        """(distance, ids on some shortest i -> j path, ids other than i and j
        on every shortest i -> j path), both ascending (apsp_query_nodes)."""
        cap = max(self.num_nodes(), 1)
        on = (ctypes.c_int32 * cap)()
        key = (ctypes.c_int32 * cap)()
        dist, n_on, n_key = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        N.check(self._lib.apsp_query_nodes(self._h, int(i), int(j), ctypes.byref(dist), on, cap, ctypes.byref(n_on),
                                           key, cap, ctypes.byref(n_key)), "apsp_query_nodes")
        return int(dist.value), list(on[: n_on.value]), list(key[: n_key.value])

    def query_paths(self, i: int, j: int) -> List[List[int]]:
        """Algorithm 8's list of shortest i -> j paths (apsp_query_paths): the
        query's path, then for every other node t on some shortest path the
        path i -> t followed by t -> j, each distinct path once.  Every path
        is shortest; the list need not hold them all.  [[i]] when i == j, []
        when j is unreachable."""
        n = max(self.num_nodes(), 1)
        ids_cap, off_cap = 8 * n, n + 1
        for _ in range(2):
            ids = (ctypes.c_int32 * ids_cap)()
            offs = (ctypes.c_int32 * off_cap)()
            dist, npaths, ids_len = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int64()
            st = self._lib.apsp_query_paths(self._h, int(i), int(j), ctypes.byref(dist), ids, ids_cap,
                                            ctypes.byref(ids_len), offs, off_cap, ctypes.byref(npaths))
            if st == N.APSP_E_CAPACITY:  # sizes reported: once more with room
                ids_cap, off_cap = int(ids_len.value), int(npaths.value) + 1
                continue
            N.check(st, "apsp_query_paths")
            return [list(ids[offs[q]:offs[q + 1]]) for q in range(npaths.value)]
        raise N.ApspError(N.APSP_E_CAPACITY, "apsp_query_paths")

    def edge_scope(self, u: int, v: int) -> Tuple[int, int]:
        r = ctypes.c_int32()
        c = ctypes.c_int32()
        N.check(self._lib.apsp_edge_scope(self._h, int(u), int(v), ctypes.byref(r), ctypes.byref(c)),
                "apsp_edge_scope")
        return int(r.value), int(c.value)

    def stats(self) -> dict:
        s = N.UpdateStats()
        N.check(self._lib.apsp_last_stats(self._h, ctypes.byref(s)), "apsp_last_stats")
        return s.as_dict()

    # -- control ----------------------------------------------------------------
    def sync(self) -> None:
        N.check(self._lib.apsp_sync(self._h), "apsp_sync")

    def set_fallback(self, policy: int, delta: float = 0.5) -> None:
        N.check(self._lib.apsp_set_fallback(self._h, int(policy), float(delta)), "apsp_set_fallback")

    def set_index_limit(self, limit: int) -> None:
        N.check(self._lib.apsp_set_index_limit(self._h, int(limit)), "apsp_set_index_limit")

    def profile(self, mask: int, every: int = 1) -> None:
        N.check(self._lib.apsp_profile_every(self._h, int(mask), int(every)), "apsp_profile_every")

    def profile_read(self, kernel: int) -> Tuple[int, float]:
        c = ctypes.c_int64()
        ms = ctypes.c_double()
        N.check(self._lib.apsp_profile_read(self._h, int(kernel), ctypes.byref(c), ctypes.byref(ms)),
                "apsp_profile_read")
        return int(c.value), float(ms.value)


def kernel_names() -> List[str]:
    lib = N.load()
    return [lib.apsp_kernel_name(k).decode() for k in range(lib.apsp_kernel_count())]


def kernel_id(name: str) -> int:
    return kernel_names().index(name)
