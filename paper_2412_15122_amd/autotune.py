"""Autotuner of the batched launch shape.

The batched launch has four knobs (apsp_batch_set_config): the schedule
(one work-group per graph from a work queue, or all graphs in lockstep with
the whole grid on every row sweep), the number of work-groups, the order in
which the work queue hands out graphs, and the loads in flight per lane.
The best choice depends on the spread of graph sizes and the number of
graphs, so the tuner times every candidate on clones of the caller's graphs
(the originals are not touched), keeps the fastest, and caches it in a JSON
file keyed by the device architecture and a coarse signature of the
workload (graph count, largest pitch and items per graph, each rounded to a
power of two).
"""
from __future__ import annotations

import json
import math
import os
from typing import Dict, List, Optional, Sequence

from .apsp import Graph, _torch
from .batch import Batch

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "paper_2412_15122_amd", "batch_tuning.json")


def _pow2(x: int) -> int:
    return 1 << max(0, math.ceil(math.log2(max(1, x))))


def arch_name() -> str:
    torch = _torch()
    return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]


def signature(graphs: Sequence[Graph], items: Sequence[tuple]) -> str:
    pmax = max((-(-g.capacity // 128)) * 128 for g in graphs) if graphs else 0
    per = len(items) / max(1, len(graphs))
    return f"g{_pow2(len(graphs))}-p{_pow2(pmax)}-i{_pow2(int(math.ceil(per)))}"


def candidates(n_cu: int, n_graphs: int) -> List[Dict[str, int]]:
    """Work-queue schedule (variants 0, 1): grid x order; lockstep schedule
    (variants 2, 3, 4): the resident grid (order does not apply)."""
    out = []
    grids = sorted({min(n_graphs, k * n_cu) for k in (1, 2, 4)} | {0})
    for variant in (0, 1):
        for order in (0, 1):
            for grid in grids:
                out.append({"grid": grid, "order": order, "variant": variant, "use_graph": 1})
    for variant in (2, 3, 4):
        out.append({"grid": 0, "order": 0, "variant": variant, "use_graph": 1})
    return out


def _load(path: str) -> dict:
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def tune(graphs: Sequence[Graph], items: Sequence[tuple], *, reps: int = 2, cache_path: Optional[str] = None,
         force: bool = False) -> dict:
    """The fastest launch config for this workload shape, from the cache or
    measured now.  Returns {"config": ..., "ms": ..., "table": [...], "cached": bool}."""
    torch = _torch()
    path = cache_path or os.environ.get("APSP_TUNING_CACHE", DEFAULT_CACHE)
    key = f"{arch_name()}:{signature(graphs, items)}"
    cache = _load(path)
    if not force and key in cache:
        ent = dict(cache[key])
        ent["cached"] = True
        ent["key"] = key
        return ent
    n_cu = torch.cuda.get_device_properties(0).multi_processor_count
    b = Batch(len(graphs), len(items))
    prep = b.prepare(graphs, items)
    table = []
    for cfg in candidates(n_cu, len(graphs)):
        b.set_config(**cfg)
        best = float("inf")
        for _ in range(max(1, reps)):
            clones = [g.clone() for g in graphs]
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            b.submit(prep, graphs=clones)
            e1.record()
            torch.cuda.synchronize()
            best = min(best, e0.elapsed_time(e1))
            for c in clones:
                c.close()
        table.append({**cfg, "ms": round(best, 4)})
    b.close()
    win = min(table, key=lambda r: r["ms"])
    ent = {"config": {k: win[k] for k in ("grid", "order", "variant", "use_graph")}, "ms": win["ms"], "table": table}
    cache[key] = ent
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        with open(path, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
    except OSError:
        pass
    out = dict(ent)
    out["cached"] = False
    out["key"] = key
    return out
