"""ctypes binding of the C ABI in include/apsp.h (argument marshalling only).

The HIP library is loaded after torch so that both share torch's HIP runtime
(the library's dependency resolves to the runtime already in the process).
There is no fallback: if the library is missing, loading raises.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libapsp.so")

APSP_INF = 1 << 30
APSP_OK = 0
APSP_E_INVALID = -1
APSP_E_NOT_FOUND = -2
APSP_E_CAPACITY = -3
APSP_E_DEVICE = -5
APSP_E_VALUE = -7
APSP_DIRECTED = 0
APSP_UNDIRECTED = 1
APSP_MINIMAX = 2      # OR-ed into the kind: minimax (bottleneck) paths
APSP_WIDEST = 4       # OR-ed into the kind: widest (maximum-capacity) paths
APSP_IMPORT_TRUSTED = 0  # apsp_import: O(n^2) checks only
APSP_IMPORT_EXACT = 1    # apsp_import: also a cold recompute, compared
APSP_FALLBACK_NEVER = 0
APSP_FALLBACK_COST = 1
APSP_FALLBACK_ALWAYS = 2
APSP_MAX_CAPACITY = 38272
APSP_BATCH_MAX_CAPACITY = 16384
APSP_NOALLOC_MAX_CAPACITY = 4224
APSP_OP_ADD_NODE = 1
APSP_OP_REMOVE_NODE = 2
APSP_OP_UPDATE_EDGE = 3
APSP_OP_QUERY = 4

STATUS_NAMES = {
    APSP_OK: "APSP_OK", APSP_E_INVALID: "APSP_E_INVALID", APSP_E_NOT_FOUND: "APSP_E_NOT_FOUND",
    APSP_E_CAPACITY: "APSP_E_CAPACITY", APSP_E_DEVICE: "APSP_E_DEVICE", APSP_E_VALUE: "APSP_E_VALUE",
}


class UpdateStats(ctypes.Structure):
    _fields_ = [
        ("flagged", ctypes.c_int64),
        ("rows", ctypes.c_int32),
        ("n_before", ctypes.c_int32),
        ("cost", ctypes.c_double),
        ("kind", ctypes.c_int32),
        ("noop", ctypes.c_int32),
        ("fallback", ctypes.c_int32),
        ("full_scans", ctypes.c_int32),
        ("sweeps", ctypes.c_int32),
        ("rows_relaxed", ctypes.c_int32),
        ("heavy_rows", ctypes.c_int32),
        ("rows_changed", ctypes.c_int32),
        ("changed", ctypes.c_int64),
        ("cost_refined", ctypes.c_double),
        ("route", ctypes.c_int32),
        ("pad", ctypes.c_int32),
    ]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class BatchItem(ctypes.Structure):
    _fields_ = [
        ("graph", ctypes.c_int32),
        ("op", ctypes.c_int32),
        ("u", ctypes.c_int32),
        ("v", ctypes.c_int32),
        ("w", ctypes.c_int32),
        ("out_cap", ctypes.c_int32),
        ("w_out_dev", ctypes.c_void_p),
        ("w_in_dev", ctypes.c_void_p),
        ("out_dev", ctypes.c_void_p),
    ]


_lib = None

# name -> (restype, argtypes)
_P = ctypes.c_void_p
_I32 = ctypes.c_int32
_I64 = ctypes.c_int64
_PI32 = ctypes.POINTER(ctypes.c_int32)
SIGNATURES = {
    "apsp_abi_version": (_I32, []),
    "apsp_last_error": (ctypes.c_char_p, []),
    "apsp_kernel_count": (_I32, []),
    "apsp_kernel_name": (ctypes.c_char_p, [_I32]),
    "apsp_required_bytes": (ctypes.c_size_t, [_I32, _I32]),
    "apsp_cold": (_I32, [_P, _I32, _I64, _I32, _I32, _P, ctypes.c_size_t, _P, ctypes.POINTER(_P)]),
    "apsp_import": (_I32, [_P, _I64, _P, _I64, _I32, _PI32, _I32, _I32, _I32, _P, ctypes.c_size_t, _P, _I32,
                           ctypes.POINTER(_P)]),
    "apsp_next_id": (_I32, [_P, _PI32]),
    "apsp_recompute_cold": (_I32, [_P]),
    "apsp_graph_destroy": (_I32, [_P]),
    "apsp_add_node": (_I32, [_P, _P, _P, _PI32]),
    "apsp_remove_node": (_I32, [_P, _I32]),
    "apsp_update_edge": (_I32, [_P, _I32, _I32, _I32]),
    "apsp_update_edge_noalloc": (_I32, [_P, _I32, _I32, _I32]),
    "apsp_noalloc_scratch_bytes": (ctypes.c_size_t, []),
    "apsp_query": (_I32, [_P, _I32, _I32, _PI32, _PI32, _I32, _PI32]),
    "apsp_query_nodes": (_I32, [_P, _I32, _I32, _PI32, _PI32, _I32, _PI32, _PI32, _I32, _PI32]),
    "apsp_read_matrix": (_I32, [_P, _P, _I64]),
    "apsp_read_adjacency": (_I32, [_P, _P, _I64]),
    "apsp_node_count": (_I32, [_P, _PI32]),
    "apsp_node_ids": (_I32, [_P, _PI32, _I32, _PI32]),
    "apsp_edge_scope": (_I32, [_P, _I32, _I32, _PI32, _PI32]),
    "apsp_query_paths": (_I32, [_P, _I32, _I32, _PI32, _PI32, _I64, ctypes.POINTER(_I64), _PI32, _I32, _PI32]),
    "apsp_last_stats": (_I32, [_P, ctypes.POINTER(UpdateStats)]),
    "apsp_sync": (_I32, [_P]),
    "apsp_set_stream": (_I32, [_P, _P]),
    "apsp_set_fallback": (_I32, [_P, _I32, ctypes.c_double]),
    "apsp_set_index_limit": (_I32, [_P, _I32]),
    "apsp_profile": (_I32, [_P, _I64]),
    "apsp_profile_every": (_I32, [_P, _I64, _I32]),
    "apsp_profile_read": (_I32, [_P, _I32, ctypes.POINTER(_I64), ctypes.POINTER(ctypes.c_double)]),
    "apsp_graph_clone": (_I32, [_P, _P, ctypes.c_size_t, _P, ctypes.POINTER(_P)]),
    "apsp_graph_relocate": (_I32, [_P, _P, ctypes.c_size_t]),
    "apsp_graph_detach": (_I32, [_P]),
    "apsp_grow": (_I32, [_P, _I32, _P, ctypes.c_size_t, _P, ctypes.POINTER(_P)]),
    "apsp_batch_workspace_bytes": (ctypes.c_size_t, [_I32, _I32]),
    "apsp_batch_create": (_I32, [_P, ctypes.c_size_t, _I32, _I32, ctypes.POINTER(_P)]),
    "apsp_batch_destroy": (_I32, [_P]),
    "apsp_batch_set_config": (_I32, [_P, _I32, _I32, _I32, _I32]),
    "apsp_batch_run": (_I32, [_P, ctypes.POINTER(_P), _I32, ctypes.POINTER(BatchItem), _I32, _P, _PI32]),
    "apsp_batch_status": (_I32, [_P]),
    "apsp_batch_phase_times": (_I32, [_P, ctypes.POINTER(ctypes.c_double), _I32, _PI32]),
    "apsp_batch_graph_times": (_I32, [_P, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double), _I32]),
}


def load():
    """Load libapsp.so (after torch, so both use one HIP runtime)."""
    global _lib
    if _lib is not None:
        return _lib
    import torch  # noqa: F401  -- puts torch's HIP runtime in the process first
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"HIP library not built: {LIB_PATH} (run __graft_entry__.build())")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


class ApspError(RuntimeError):
    def __init__(self, status: int, where: str):
        msg = load().apsp_last_error().decode(errors="replace")
        super().__init__(f"{where}: {STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def check(status: int, where: str) -> None:
    if status != APSP_OK:
        raise ApspError(status, where)
