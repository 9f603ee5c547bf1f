"""Re-run of the paper's warm/cold time ratios (its Experiments I-IV, Tables
1-4) with the CPU procedures of procedures.c, one thread each, on the host
that runs it.  Benchmark infrastructure: it shares no code with the HIP
library and does not use the oracle (its cold starts are procedures.c's own).

Workload: undirected complete graphs with symmetric weights uniform on
[1, wmax] (10000 by default; the paper does not state its weights), a random node removed
(Algorithm 5 and Algorithm 11 against Floyd-Warshall on G - G_k), a random
edge set to a new uniform weight (Algorithm 6 against Floyd-Warshall on G'),
random pairs queried (Algorithm 7 against Dijkstra on G).  delta = 1 (the
warm branch always; the paper's delta is not stated), so the ratio measures
the warm procedure itself; the mean Cost is reported beside it.  Every warm
result is checked against its cold counterpart.

    python -m paper_cpu.tables --sizes 1000,2000,3000 --repeats 5
"""
from __future__ import annotations

import argparse
import json
import os
import sys

import numpy as np

from . import procedures as PC

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
from paper_2412_15122_amd import workloads as W  # noqa: E402  (seeded generators only)


def one_size(n: int, repeats: int, queries: int, seed: int, wmax: int) -> dict:
    rng = np.random.default_rng(seed + n)
    r_rm, r_ed, r_q, r_key, costs, refined = [], [], [], [], [], []
    for rep in range(repeats):
        A = W.symmetric_complete_graph(n, 1, wmax, seed=int(rng.integers(1 << 30)))
        D, _ = PC.fw(A)
        # Experiment I and IV: remove a random node
        k = int(rng.integers(n))
        keep = [x for x in range(n) if x != k]
        Dk_cold, t_cold = PC.fw(np.ascontiguousarray(A[np.ix_(keep, keep)]))
        print(f"n={n} rep={rep}: cold Floyd-Warshall of G - G_k {t_cold:.2f} s", flush=True)
        Dk, s5 = PC.remove(A, D, k, 1.0)
        print(f"n={n} rep={rep}: Algorithm 5 {s5['seconds']:.2f} s", flush=True)
        Dk11, s11 = PC.remove_key(A, D, k, 1.0)
        print(f"n={n} rep={rep}: Algorithm 11 {s11['seconds']:.2f} s", flush=True)
        assert np.array_equal(Dk, Dk_cold) and np.array_equal(Dk11, Dk_cold)
        r_rm.append(s5["seconds"] / t_cold)
        r_key.append(s11["seconds"] / t_cold)
        costs.append(s5["cost"])
        refined.append(s11["phi"] / max(s5["phi"], 1))
        # Experiment II: set a random edge to a new weight
        u, v = (int(x) for x in rng.choice(n, size=2, replace=False))
        w = int(rng.integers(1, wmax + 1))
        A2 = A.copy()
        A2[u, v] = A2[v, u] = w
        De_cold, t_cold_e = PC.fw(A2)
        print(f"n={n} rep={rep}: cold Floyd-Warshall of G' {t_cold_e:.2f} s", flush=True)
        De, se = PC.edge(A, D, u, v, w, 1.0, True)
        assert np.array_equal(De, De_cold)
        r_ed.append(se["seconds"] / t_cold_e)
        # Experiment III: single-pair queries
        tw = tc = 0.0
        for _ in range(queries):
            i, j = (int(x) for x in rng.integers(0, n, size=2))
            d1, _, t1 = PC.query(A, D, i, j)
            d2, _, t2 = PC.dijkstra_path(A, i, j)
            assert d1 == d2
            tw += t1
            tc += t2
        r_q.append(tw / tc)
        print(f"n={n} rep={rep}: remove {r_rm[-1]:.3f} edge {r_ed[-1]:.3f} query {r_q[-1]:.4f} "
              f"remove-key {r_key[-1]:.3f} cost {costs[-1]:.3f} phi'/phi {refined[-1]:.3f} "
              f"(cold FW {t_cold:.2f} s)", flush=True)

    def ms(x):
        return [round(float(np.mean(x)), 3), round(float(np.std(x)), 3)]
    return {"n": n, "wmax": wmax, "repeats": repeats, "remove": ms(r_rm), "edge": ms(r_ed), "query": ms(r_q),
            "remove_key": ms(r_key), "cost": ms(costs), "phi_refined_over_phi": ms(refined)}


def main() -> None:
    ap = argparse.ArgumentParser()
    ap.add_argument("--sizes", default="1000,2000,3000")
    ap.add_argument("--repeats", type=int, default=5)
    ap.add_argument("--queries", type=int, default=200)
    ap.add_argument("--seed", type=int, default=2412)
    ap.add_argument("--wmax", type=int, default=10000, help="weights uniform on [1, wmax]")
    ap.add_argument("--json", default="")
    a = ap.parse_args()
    rows = [one_size(int(s), a.repeats, a.queries, a.seed, a.wmax) for s in a.sizes.split(",")]
    print("| N | remove (Alg. 5) | edge (Alg. 6) | query (Alg. 7) | remove (Alg. 11) | Cost | Phi'/Phi |")
    print("|---|---|---|---|---|---|---|")
    for r in rows:
        f = lambda p: f"{p[0]:.3f} ± {p[1]:.3f}"  # noqa: E731
        print(f"| {r['n']} | {f(r['remove'])} | {f(r['edge'])} | {f(r['query'])} | {f(r['remove_key'])} "
              f"| {f(r['cost'])} | {f(r['phi_refined_over_phi'])} |")
    if a.json:
        with open(a.json, "w") as fh:
            json.dump(rows, fh, indent=1)


if __name__ == "__main__":
    main()
