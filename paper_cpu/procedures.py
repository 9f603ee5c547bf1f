"""The paper's own warm-start procedures on the CPU -- TEST AND BENCHMARK
INFRASTRUCTURE ONLY.

Thin ctypes wrappers over ``procedures.c`` (one thread, the steps of
Algorithms 5, 6, 7 and 11 in the paper's order, with textbook Floyd-Warshall
and dense Dijkstra as the cold starts they are compared with).  Only `tests/`
and the benchmark's CPU baseline leg use it; it shares no code with the HIP
library.  Matrices are int32 with INF = 2**30, row-major.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import time
from typing import List, Tuple

import numpy as np

INF = 1 << 30

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "procedures.c")
_LIB = os.path.join(_HERE, "libpaper_cpu.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile with gcc, one thread, portable x86-64-v2 code."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O3", "-march=x86-64-v2", "-shared", "-fPIC", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        i32, p, f64 = ctypes.c_int32, ctypes.c_void_p, ctypes.c_double
        sig = {
            "pc_fw": [i32, p, p],
            "pc_remove": [i32, p, p, i32, f64, p, p, p],
            "pc_remove_key": [i32, p, p, i32, f64, p, p, p],
            "pc_edge": [i32, p, p, i32, i32, i32, i32, f64, p, p],
            "pc_query": [i32, p, p, i32, i32, p, p, p],
            "pc_dijkstra_path": [i32, p, i32, i32, p, p, p],
            "pc_remove_sample": [i32, p, p, i32, i32, p],
        }
        for name, args in sig.items():
            f = getattr(lib, name)
            f.argtypes = args
            f.restype = ctypes.c_int
        _lib = lib
    return _lib


def _mat(A) -> np.ndarray:
    A = np.ascontiguousarray(A, dtype=np.int32)
    assert A.ndim == 2 and A.shape[0] == A.shape[1]
    return A


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _ok(rc: int, what: str) -> None:
    if rc != 0:
        raise MemoryError(f"{what}: out of host memory")


def fw(A) -> Tuple[np.ndarray, float]:
    """Cold start: (M_G, seconds)."""
    A = _mat(A)
    D = np.empty_like(A)
    t0 = time.perf_counter()
    _ok(_load().pc_fw(A.shape[0], _p(A), _p(D)), "pc_fw")
    return D, time.perf_counter() - t0


def _removal(fn, A, D, k, delta):
    A, D = _mat(A), _mat(D)
    n = A.shape[0]
    D2 = np.empty((n - 1, n - 1), dtype=np.int32)
    st = np.zeros(5, dtype=np.int64)
    cost = ctypes.c_double()
    t0 = time.perf_counter()
    _ok(fn(n, _p(A), _p(D), int(k), float(delta), _p(D2), _p(st), ctypes.byref(cost)), "removal")
    dt = time.perf_counter() - t0
    return D2, {"phi": int(st[0]), "listed": int(st[1]), "fell_back": bool(st[2]), "dijkstra_runs": int(st[3]),
                "flagged": int(st[4]), "cost": float(cost.value), "seconds": dt}


def remove(A, D, k: int, delta: float):
    """Algorithm 5: (M_{G - G_k} in the order of the remaining nodes, stats)."""
    return _removal(_load().pc_remove, A, D, k, delta)


def remove_key(A, D, k: int, delta: float):
    """Algorithm 11 (key_node_list-refined need_update_list, then Algorithm
    5 from its Cost step).  stats['flagged'] is the unrefined count."""
    return _removal(_load().pc_remove_key, A, D, k, delta)


def edge(A, D, u: int, v: int, w: int, delta: float, undirected: bool):
    """Algorithm 6: (M_{G'}, stats) with edge u -> v (and v -> u when
    undirected) set to w."""
    A, D = _mat(A), _mat(D)
    n = A.shape[0]
    out = np.empty_like(D)
    st = np.zeros(5, dtype=np.int64)
    t0 = time.perf_counter()
    _ok(_load().pc_edge(n, _p(A), _p(D), int(undirected), int(u), int(v), int(w), float(delta), _p(out), _p(st)),
        "pc_edge")
    dt = time.perf_counter() - t0
    return out, {"phi": int(st[0]), "listed": int(st[1]), "fell_back": bool(st[2]), "dijkstra_runs": int(st[3]),
                 "removed": int(st[4]), "seconds": dt}


def query(A, D, i: int, j: int) -> Tuple[int, List[int], float]:
    """Algorithm 7: (distance, path, seconds)."""
    A, D = _mat(A), _mat(D)
    n = A.shape[0]
    path = np.empty(max(n, 1), dtype=np.int32)
    ln, dist = ctypes.c_int32(), ctypes.c_int32()
    t0 = time.perf_counter()
    _ok(_load().pc_query(n, _p(A), _p(D), int(i), int(j), _p(path), ctypes.byref(ln), ctypes.byref(dist)),
        "pc_query")
    dt = time.perf_counter() - t0
    return int(dist.value), path[: ln.value].tolist(), dt


def dijkstra_path(A, i: int, j: int) -> Tuple[int, List[int], float]:
    """Cold single-pair query: (distance, path, seconds)."""
    A = _mat(A)
    n = A.shape[0]
    path = np.empty(max(n, 1), dtype=np.int32)
    ln, dist = ctypes.c_int32(), ctypes.c_int32()
    t0 = time.perf_counter()
    _ok(_load().pc_dijkstra_path(n, _p(A), int(i), int(j), _p(path), ctypes.byref(ln), ctypes.byref(dist)),
        "pc_dijkstra_path")
    dt = time.perf_counter() - t0
    return int(dist.value), path[: ln.value].tolist(), dt


def remove_sample(A, D, k: int, max_runs: int) -> dict:
    """Bounded timing sample of Algorithm 5: the need_update_list step in
    full, then the first `max_runs` Dijkstra runs; the whole removal's time
    extrapolated as list time + Phi x mean run time."""
    A, D = _mat(A), _mat(D)
    n = A.shape[0]
    st = np.zeros(5, dtype=np.int64)
    _ok(_load().pc_remove_sample(n, _p(A), _p(D), int(k), int(max_runs), _p(st)), "pc_remove_sample")
    phi, listed, runs, ns_lists, ns_runs = (int(x) for x in st)
    per_run = ns_runs / max(runs, 1) * 1e-9
    return {"phi": phi, "listed": listed, "runs_timed": runs, "list_s": ns_lists * 1e-9, "per_run_s": per_run,
            "removal_s": ns_lists * 1e-9 + phi * per_run}
