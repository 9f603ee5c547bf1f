"""Benchmark: warm-start APSP updates on one MI355X.

Workload: undirected complete graph, n = 16384, symmetric int32 weights
U[1, 10000] (D = 1 GiB).  One step = 1000 updates applied in sequence
(300 add-node / 200 remove-node / 250 edge decrease / 250 edge increase,
seeded shuffle; the first is the worst-case increase: among the 64 lightest
edges, the one with the largest |R| * |C|, raised to 20000) to the n-node
graph, which is restored from a device snapshot before every step, outside
the timed region.  Every input (graph, add-node weight vectors) is resident
in HBM before the timed region.  The same line also carries the batched
workload (512 graphs x 8 updates in one persistent launch against one call
per update) and the served one (64 resident graphs, Poisson requests, p50 /
p99 against the plain path).  Prints one JSON line.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--n 16384]
                  [--no-cpu-baseline] [--no-verify] [--legs batched,serving]
  python bench.py --workload batched | serving | kernels   (one workload alone)
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0        # MI355X HBM3E, 8 TB/s
N_DEFAULT = 16384


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=N_DEFAULT)
    ap.add_argument("--updates", type=int, default=1000, help="updates per step (multiple of 20)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-verify", action="store_true")
    ap.add_argument("--cold-reps", type=int, default=3)
    ap.add_argument("--trace", action="store_true", help="log per-update mask statistics during warmup")
    ap.add_argument("--mix", default="all", choices=["all", "add", "remove", "decrease", "increase"],
                    help="update kinds of a step (profiling runs of one kind); 'all' is the benchmark mix")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first run a plain 1 GiB device copy three times (counter calibration)")
    ap.add_argument("--workload", default="updates", choices=["updates", "batched", "serving", "kernels"],
                    help="updates: the n=16384 update stream (default); batched: 512 graphs with 8 queued "
                         "updates each, one persistent launch vs one call per update; kernels: standalone "
                         "medians of single updates on the n=16384 graph (add, remove, a forced wide edge "
                         "decrease and the worst-case increase that undoes it)")
    ap.add_argument("--reps", type=int, default=20, help="kernels: repetitions per update kind")
    ap.add_argument("--prof-every", type=int, default=10,
                    help="updates: HIP events bracket launches 0, k, 2k, ... of the dominant kernel in each timed "
                         "step (two event records cost ~11 us of stream time; the launches between carry none)")
    ap.add_argument("--reps-sweep", type=int, default=5,
                    help="updates: repetitions of the edge-sweep roofline probe (forced decrease, worst increase)")
    ap.add_argument("--graphs", type=int, default=None, help="batched / serving: number of graphs (512 / 64)")
    ap.add_argument("--batch-config", default=None,
                    help="batched: grid,order,variant to use instead of autotuning")
    ap.add_argument("--rates", default="1000,3000,10000,30000,100000",
                    help="serving: Poisson arrival rates (requests/s) to sweep")
    ap.add_argument("--requests", type=int, default=20000, help="serving: requests per rate")
    ap.add_argument("--legs", default="batched,serving",
                    help="updates workload: further legs reported in the same line ('' for none)")
    ap.add_argument("--leg-rates", default="10000,100000", help="serving leg: arrival rates (req/s)")
    ap.add_argument("--schedules", default="lockstep,hybrid",
                    help="serving: server schedules to run (the first is the reported one)")
    ap.add_argument("--semiring", default="shortest", choices=["shortest", "minimax"],
                    help="updates: shortest paths (the benchmark) or minimax (bottleneck) paths")
    ap.add_argument("--fallback", type=float, default=None,
                    help="updates: Algorithm 5's cost fallback with this delta (default: never)")
    ap.add_argument("--small-batch", type=int, default=None,
                    help="serving: queued requests the lockstep server sends as single calls (default: the server's)")
    return ap.parse_args()


# ---------------------------------------------------------------------------
# algorithmic bytes per launch of the sweep kernels
# ---------------------------------------------------------------------------
# The benchmark graph is undirected, so D is symmetric and each sweep needs
# one entry per unordered pair (see sweep_bytes): add_relax reads every pair
# of old nodes once, 4 n (n - 1) / 2 bytes per added node, n the live count
# before the add; mask_detect (a removal; an edge increase's mask runs in
# edge_sweep) every pair of the other n - 1 nodes, 4 (n - 1)(n - 2) / 2
# bytes.  Writes (changed entries and their mirrors, the flag bitmap) are not
# counted.


KERNEL_SOURCES = ("update.hip", "device_common.h")   # where add_relax and mask_detect live


def source_hash():
    """Hash of the sweep kernels' sources: counter figures taken on other
    sources are not reported."""
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2412_15122_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def sweep_bytes(kind, live, count_only=False):
    """Algorithmic bytes of one full sweep of D on the undirected graph of
    `live` nodes.  D is symmetric, so an addition's relaxation (Theorem 3,
    in = out) reads each unordered pair of the old nodes once, 4 n (n-1) / 2
    bytes, and a removal's mask (Corollary 3) each unordered pair of the
    other n - 1 nodes, 4 (n-1)(n-2) / 2.  count_only: the count-only mask of
    a minimax removal's spanning-forest route, which reads the rows of the
    other n - 1 nodes in full, 4 (n-1) n."""
    if kind == "add":
        return 2 * live * (live - 1)
    if count_only:
        return 4 * (live - 1) * live
    return 2 * (live - 1) * (live - 2)


def traffic_from_profiles(kernel):
    """HBM bytes per launch of `kernel` from the committed counter summary,
    or None when it was taken on other sources."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    ent = rec.get(kernel)
    if not ent or ent.get("source_hash") != source_hash():
        return None
    return ent.get("bytes_per_launch")


# ---------------------------------------------------------------------------
# CPU baseline: the oracle's cold Floyd-Warshall, sampled
# ---------------------------------------------------------------------------

def cpu_baseline(adj, budget_s=12.0):
    from oracle import oracle as O
    n = adj.shape[0]
    D = O.fw_init(adj)
    threads = O.max_threads()
    done = 0
    t0 = time.perf_counter()
    chunk = 4
    while done < n and time.perf_counter() - t0 < budget_s:
        k1 = min(n, done + chunk)
        O.fw_pivots(D, done, k1, threads)
        done = k1
        chunk = min(64, chunk * 2)
    el = time.perf_counter() - t0
    per_pivot = el / done
    full = per_pivot * n
    return {
        "value": 1.0 / full,
        "unit": "updates/s",
        "cores": threads,
        "kind": "oracle",
        "sample": (f"textbook Floyd-Warshall (the oracle's cold recompute of one updated graph) at n={n}: "
                   f"pivots 0..{done - 1} of {n} timed ({el:.1f} s, {per_pivot * 1e3:.1f} ms/pivot), "
                   f"extrapolated to the full {n} pivots = {full:.0f} s per update"),
    }


def cpu_context(adj):
    """Further oracle timings on the host, context beside the baseline (a few
    seconds): cold Floyd-Warshall of the n = 256 directed complete graph on
    one thread (median of 5); of a directed n = 4096 graph of 95% density on
    one thread and on all, sampled by pivots and extrapolated; one dense
    Dijkstra row of the n = 16384 graph on one thread."""
    from oracle import oracle as O
    from paper_2412_15122_amd import workloads as W
    out = {"host_cpu": "unknown", "logical_cpus": os.cpu_count(), "threads": O.max_threads()}
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    out["host_cpu"] = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    a256 = W.random_graph(256, 1, 1000, undirected=False, density=1.0, seed=W.seed_for(1))
    ts = []
    for _ in range(5):
        t = time.perf_counter()
        O.fw(a256, threads=1)
        ts.append(time.perf_counter() - t)
    out["fw_n256_1thread_ms"] = round(1e3 * float(np.median(ts)), 2)
    a4096 = W.random_graph(4096, 1, 10000, undirected=False, density=0.95, seed=W.seed_for(2))
    for label, threads, pivots in (("1thread", 1, 32), ("all_threads", O.max_threads(), 128)):
        D = O.fw_init(a4096)
        t = time.perf_counter()
        O.fw_pivots(D, 0, pivots, threads)
        el = time.perf_counter() - t
        out[f"fw_n4096_{label}_s"] = round(el / pivots * 4096, 2)
    t = time.perf_counter()
    O.dijkstra_rows(adj, [0, 1], threads=1)
    out["dijkstra_row_n16384_1thread_ms"] = round(1e3 * (time.perf_counter() - t) / 2, 1)
    out["note"] = ("n=4096 figures extrapolated from 32 (one thread) and 128 (all threads) timed pivots; "
                   "context only, not the baseline")
    return out


# ---------------------------------------------------------------------------
# main
# ---------------------------------------------------------------------------

def batch_items(wls, W):
    items = []
    for gi, w in enumerate(wls):
        for up in w.updates:
            if up.kind == W.ADD:
                items.append(("add", gi, up.w_out, up.w_in))
            elif up.kind == W.REMOVE:
                items.append(("remove", gi, up.u))
            else:
                items.append(("edge", gi, up.u, up.v, up.w))
    return items


def bench_batched(args):
    import torch
    torch.cuda.set_device(0)
    out = batched_leg(args.graphs or 512, args.warmup, args.steps, args.batch_config)
    print(json.dumps(out), flush=True)


def batched_leg(graphs, warmup, steps, batch_config=None):
    """512 directed complete graphs (n log-uniform in [128, 2048]), 8 queued
    updates each: one autotuned, graph-replayed persistent launch against the
    plain path (one library call, i.e. one set of kernel launches, per
    update).  Each timed run starts from fresh device copies of the same
    cold-started graphs; the two paths' final matrices are compared."""
    import torch
    from paper_2412_15122_amd import workloads as W
    from paper_2412_15122_amd.apsp import Graph
    from paper_2412_15122_amd.batch import Batch
    from paper_2412_15122_amd import autotune
    t = time.perf_counter()
    wls = W.config4(graphs=graphs)
    log(f"[bench] {len(wls)} graphs generated in {time.perf_counter() - t:.1f}s")
    base = [Graph(w.adj, undirected=False, capacity=w.adj.shape[0] + 8) for w in wls]
    torch.cuda.synchronize()
    items = batch_items(wls, W)
    n_upd = len(items)
    ns = np.array([w.adj.shape[0] for w in wls])
    log(f"[bench] cold starts done; {n_upd} updates; sum n^2 = {int((ns.astype(np.int64) ** 2).sum())}")
    if batch_config:
        gr, od, va = (int(x) for x in batch_config.split(","))
        tuned = {"config": {"grid": gr, "order": od, "variant": va, "use_graph": 1}, "ms": None, "table": [],
                 "key": "fixed"}
    else:
        tuned = autotune.tune(base, items, reps=2, force=True)
    cfg = tuned["config"]
    log(f"[bench] autotuned config {cfg} ({tuned['ms']} ms); table: " +
        ", ".join(f"g{r['grid']}/o{r['order']}/v{r['variant']}={r['ms']}" for r in tuned["table"]))
    b = Batch(len(base), n_upd, **cfg)
    prep = b.prepare(base, items)

    # staged device weights for the plain path (resident before timing)
    dev_w = []
    for it in items:
        if it[0] == "add":
            dev_w.append((torch.from_numpy(np.ascontiguousarray(it[2])).cuda(),
                          torch.from_numpy(np.ascontiguousarray(it[3])).cuda()))
        else:
            dev_w.append(None)

    def plain(gs):
        for t, it in enumerate(items):
            g = gs[it[1]]
            if it[0] == "add":
                g.add_node_device(dev_w[t][0].data_ptr(), dev_w[t][1].data_ptr())
            elif it[0] == "remove":
                g.remove_node(it[2])
            else:
                g.update_edge(it[2], it[3], it[4])

    batched_ms, plain_ms, verify = [], [], True
    for rep in range(warmup + steps):
        ga = [g.clone() for g in base]
        gb = [g.clone() for g in base]
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        e0.record()
        b.submit(prep, graphs=ga)
        e1.record()
        torch.cuda.synchronize()
        tb = (time.perf_counter() - t0) * 1e3
        st_us, en_us = b.graph_times(len(base))
        dur = en_us - st_us
        big = int(np.argmax(ns))
        spans = {"makespan_us": round(float(en_us.max()), 1), "max_graph_us": round(float(dur.max()), 1),
                 "mean_graph_us": round(float(dur.mean()), 1), "largest_graph_us": round(float(dur[big]), 1),
                 "largest_graph_n": int(ns[big]), "last_start_us": round(float(st_us.max()), 1)}
        log(f"[bench] per-graph spans: {spans}")
        if cfg["variant"] >= 2 and rep == 0:
            ph = b.phase_times()
            log("[bench] lockstep phase ends (us): " + " ".join(f"{x:.0f}" for x in ph))
            try:
                b.status()
                log("[bench] lockstep barriers: ok")
            except Exception as exc:  # reported, the run continues
                log(f"[bench] lockstep barriers: {exc}")
        if rep == 0:
            for gi in np.argsort(-dur)[:6]:
                log(f"[bench]   slow graph {gi}: n={ns[gi]} {dur[gi]:.0f} us, updates "
                    + " ".join(u.kind for u in wls[gi].updates))
        t0 = time.perf_counter()
        e2, e3 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e2.record()
        plain(gb)
        e3.record()
        torch.cuda.synchronize()
        tp = (time.perf_counter() - t0) * 1e3
        same = all(torch.equal(x.matrix_device("D"), y.matrix_device("D")) for x, y in zip(ga, gb))
        verify = verify and same
        log(f"[bench] rep {rep}: batched {tb:.2f} ms wall ({e0.elapsed_time(e1):.2f} ms events), "
            f"plain {tp:.1f} ms wall ({e2.elapsed_time(e3):.1f} ms events), equal={same}")
        if rep >= warmup:
            batched_ms.append(tb)
            plain_ms.append(tp)
        for x in ga + gb:
            x.close()
    bt, pt = float(np.median(batched_ms)), float(np.median(plain_ms))
    # algorithmic bytes: one read of D per add (relaxation) and per removal
    # (mask); live counts replayed per graph
    alg = 0
    for gi, w in enumerate(wls):
        live = w.adj.shape[0]
        for up in w.updates:
            if up.kind == W.ADD:
                alg += 4 * live * live
                live += 1
            elif up.kind == W.REMOVE:
                alg += 4 * (live - 1) * live
                live -= 1
    achieved = alg / (bt * 1e-3) / 1e9
    out = {
        "metric": "batched warm-start APSP updates/s (512 graphs x 8 updates, 1 GPU)",
        "value": round(n_upd / (bt * 1e-3), 1),
        "unit": "updates/s",
        "n_gpus": 1, "steps": steps, "warmup": warmup,
        "ms_per_step": round(bt, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "i32", "data": "synthetic",
        "config": {"workload": (f"{len(wls)} directed complete graphs, n log-uniform in [128, 2048], weights "
                                f"U[1,5000], {n_upd} queued updates (8 per graph), one persistent launch"),
                   "graphs": len(wls), "updates_per_step": n_upd, "parallelism": "none (1 GPU)",
                   "launch": cfg},
        "plain_path": {"ms_per_step": round(pt, 2), "updates_per_s": round(n_upd / (pt * 1e-3), 1),
                       "what": "one library call (its kernel launches) per update, same updates"},
        "batched_vs_plain_speedup": round(pt / bt, 2),
        "per_graph_spans": spans,
        "verified_vs_plain": verify,
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None, "kernel": "k_batch (whole launch)",
                     "algorithmic_bytes_per_launch": alg},
        "autotune": {"key": tuned["key"], "table": tuned["table"]},
    }
    b.close()
    for g in base:
        g.close()
    return out


def bench_serving(args):
    import torch
    torch.cuda.set_device(0)
    out = serving_leg(args.graphs or 64, [float(x) for x in args.rates.split(",")], args.requests,
                      args.schedules.split(","), args.small_batch)
    print(json.dumps(out), flush=True)


def serving_leg(graphs, rates, requests, schedules, small_batch=None):
    """64 resident directed complete graphs (n uniform in [1024, 8192]),
    Poisson requests (45% increase, 45% decrease, 2.5% add, 2.5% remove, 5%
    query) swept over arrival rates: the continuous-batching server against
    the plain path (one library call per request, no batching).  Graphs are
    cold-started before each timed run; every request's latency is its
    completion time (event observed) minus its arrival time."""
    import torch
    from paper_2412_15122_amd import workloads as W
    from paper_2412_15122_amd import serve
    from paper_2412_15122_amd.apsp import Graph
    t = time.perf_counter()
    adjs = W.config5_graphs(graphs=graphs)
    ns = [a.shape[0] for a in adjs]
    log(f"[bench] {len(adjs)} graphs generated in {time.perf_counter() - t:.1f}s; n {min(ns)}..{max(ns)}")
    rows = []
    for rate in rates:
        per = {}
        for sched in schedules:
            gen = W.Config5Requests(adjs)
            reqs = serve.requests_from_stream(gen, rate, requests)
            kw = {} if small_batch is None else {"small_batch": small_batch}
            srv = serve.Server(adjs, streams=4, schedule=sched, **kw)
            srv.preload()
            r = srv.run(reqs)
            r["stats"] = dict(srv.stats)
            srv.close()
            del srv
            torch.cuda.empty_cache()
            per[sched] = r
            log(f"[bench] rate {rate:.0f}/s {sched}: {r['updates_per_s']:.0f} upd/s p50 {r['p50_ms']:.3f} ms "
                f"p99 {r['p99_ms']:.3f} ms {r['stats']}")
        s = per[schedules[0]]
        gs = [Graph(a, capacity=a.shape[0] + 64) for a in adjs]
        torch.cuda.synchronize()
        p = serve.serve_plain(gs, reqs)
        for g in gs:
            g.close()
        del gs
        torch.cuda.empty_cache()
        rnd = lambda d: {k: (round(v, 4) if isinstance(v, float) else v) for k, v in d.items()}
        row = {"rate": rate, "served": rnd(s), "plain": rnd(p)}
        for sched in schedules[1:]:
            row[sched] = rnd(per[sched])
        rows.append(row)
        log(f"[bench] rate {rate:.0f}/s: plain {p['updates_per_s']:.0f} upd/s p50 {p['p50_ms']:.3f} "
            f"p99 {p['p99_ms']:.3f} ms")
    top = rows[-1]
    out = {
        "metric": "served warm-start APSP updates/s (64 resident graphs, 1 GPU)",
        "value": round(top["served"]["updates_per_s"], 1),
        "unit": "updates/s",
        "n_gpus": 1, "steps": len(rates), "warmup": 0,
        "ms_per_step": round(top["served"]["wall_s"] * 1e3, 2),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "i32", "data": "synthetic",
        "config": {"workload": (f"{len(adjs)} directed complete graphs, n uniform in [1024, 8192], weights U[1,10000]; "
                                f"Poisson requests, {requests} per rate: 45% increase, 45% decrease, 2.5% add, "
                                f"2.5% remove, 5% single-pair query"),
                   "graphs": len(adjs), "parallelism": "none (1 GPU)", "rates": rates,
                   "schedule": schedules[0]},
        "latency_ms": {"p50": top["served"]["p50_ms"], "p99": top["served"]["p99_ms"]},
        "plain_path": {"updates_per_s": round(top["plain"]["updates_per_s"], 1), "p50_ms": top["plain"]["p50_ms"],
                       "p99_ms": top["plain"]["p99_ms"]},
        "sweep": rows,
    }
    return out


def bench_kernels(args):
    """Standalone medians of single updates on the undirected complete graph
    n = 16384 (every repetition starts from the same distances):
      decrease the most used of the 64 lightest edges lowered to 0: the
               relaxation sweeps nearly every row in one of the two
               directions (a forced wide K1 sweep), then
      increase the same edge back to its weight: the worst-case tight
               increase (mask over R x C, then the recompute);
      remove   a random live node, then
      add      the same node back (its original weights, now the newest id).
    Times are HIP events on the graph's stream around each call."""
    import torch
    from paper_2412_15122_amd import workloads as W
    from paper_2412_15122_amd.apsp import Graph
    n = args.n
    adj = W.config3_graph(n)
    g = Graph(adj, undirected=True, capacity=n + 8)
    torch.cuda.synchronize()
    log(f"[bench] cold start done (n={n})")
    rng = np.random.default_rng(2412151223)
    orig = {i: i for i in range(n)}          # id -> row of adj (weights of the node)
    live = list(range(n))
    times = {"remove": [], "add": [], "decrease": [], "increase": []}
    stats = {"remove": [], "add": [], "decrease": [], "increase": []}

    def timed(kind, fn):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        out = fn()
        e1.record()
        torch.cuda.synchronize()
        times[kind].append(e0.elapsed_time(e1))
        stats[kind].append(g.stats())
        return out

    cands = W.lightest_edges(adj, 64, True)
    best, best_key = None, None
    for (u, v, wt) in cands:
        r, c = g.edge_scope(u, v)
        key = (-(r * c), u, v)
        if best_key is None or key < best_key:
            best, best_key = (u, v, wt, r, c), key
    u, v, wt, r0, c0 = best
    log(f"[bench] worst-case edge ({u},{v}) weight {wt}: |R|={r0} |C|={c0}")
    for rep in range(args.reps):
        timed("decrease", lambda: g.update_edge(u, v, 0))
        timed("increase", lambda: g.update_edge(u, v, wt))
    for rep in range(args.reps):
        k = live[int(rng.integers(len(live)))]
        timed("remove", lambda: g.remove_node(k))
        live.remove(k)
        w = torch.from_numpy(np.ascontiguousarray(adj[orig[k], [orig[x] for x in live]], dtype=np.int32)).cuda()
        torch.cuda.synchronize()
        nid = timed("add", lambda: g.add_node_device(w.data_ptr(), w.data_ptr()))
        orig[nid] = orig.pop(k)
        live.append(nid)
    out = {"n": n, "reps": args.reps, "edge": [int(u), int(v), int(wt)], "edge_scope": [int(r0), int(c0)]}
    for kind in times:
        t = np.array(times[kind])
        st = stats[kind]
        row = {"median_ms": round(float(np.median(t)), 4), "p90_ms": round(float(np.percentile(t, 90)), 4),
               "min_ms": round(float(t.min()), 4)}
        if kind in ("decrease", "add"):
            rr = float(np.median([s_["rows_relaxed"] for s_ in st]))
            row["rows_relaxed"] = rr
            # bytes swept over the median time of the whole call: a decrease reads its rows
            # (4 n bytes each); an addition to the undirected graph reads each unordered
            # pair of the old nodes once (D is symmetric)
            swept = rr * 4 * n if kind == "decrease" else sweep_bytes("add", n)
            row["swept_GBps_whole_call"] = round(swept / (float(np.median(t)) * 1e-3) / 1e9, 1)
        if kind in ("remove", "increase"):
            row["flagged"] = float(np.median([s_["flagged"] for s_ in st]))
            row["rows"] = float(np.median([s_["rows"] for s_ in st]))
            row["changed"] = float(np.median([s_["changed"] for s_ in st]))
        out[kind] = row
        log(f"[bench] {kind}: {row}")
    ok = None if args.no_verify else bool(np.array_equal(g.matrix(), _cold_matrix(g)))
    log(f"[bench] final matrix equals a cold recompute: {ok}")
    out["verified_vs_gpu_cold"] = ok
    print(json.dumps({"workload": "kernels", **out}), flush=True)
    return 0 if ok is not False else 1


def edge_sweep_roofline(base, worst, adj, kid, reps):
    """The edge update's sweep kernel against HBM, on a copy of the n-node
    graph: the stream's worst-case edge lowered to 0 (a forced wide
    decrease: rows_relaxed rows are read, 4n bytes each) and raised back to
    its weight (the tight increase's mask: with the edge at 0, u and v are
    equally far from every node, so both pair tests hold on every row; the
    mask of an undirected graph is symmetric, so a tested row i reads its
    columns j > i, 4 (n - 1 - i) bytes).  Average kernel time per launch by
    HIP events on the graph's stream."""
    import torch
    u, v = int(worst[0]), int(worst[1])
    wt = int(adj[u, v])
    h = base.clone()
    n = len(h.ids())
    out = {}
    for kind, w in (("decrease", 0), ("increase", wt)):
        out[kind] = {"ms": [], "rows": [], "bytes": []}
    for _ in range(reps):
        for kind, w in (("decrease", 0), ("increase", wt)):
            if kind == "increase":
                D = h.matrix_device("D")
                tested = torch.nonzero(D[:n, u] == D[:n, v]).flatten().to(torch.int64)
                rows_read = int(tested.numel())
                upper_bytes = int((4 * (n - 1 - tested)).sum().item())
                del D, tested
            h.profile(1 << kid["edge_sweep"])
            h.update_edge(u, v, w)
            torch.cuda.synchronize()
            c, ms = h.profile_read(kid["edge_sweep"])
            h.profile(0)
            st = h.stats()
            out[kind]["ms"].append(ms / max(c, 1))
            out[kind]["rows"].append(st["rows_relaxed"] if kind == "decrease" else rows_read)
            out[kind]["bytes"].append(4 * n * st["rows_relaxed"] if kind == "decrease" else upper_bytes)
    h.close()
    res = {"edge": [u, v, wt], "n": n}
    for kind, d in out.items():
        ms = float(np.median(d["ms"]))
        rows = float(np.median(d["rows"]))
        nbytes = float(np.median(d["bytes"]))
        gbs = nbytes / (ms * 1e-3) / 1e9
        res[kind] = {"avg_launch_ms": round(ms, 4), "rows_read": rows, "bytes": int(nbytes),
                     "achieved": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4)}
    log(f"[bench] edge sweep: {res}")
    return res


def _cold_matrix(g):
    c = g.clone()
    c.recompute_cold()
    m = c.matrix()
    c.close()
    return m


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the hot path is single-GPU by design "
              "(multi-GPU sharding is described, not built); run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    if args.workload == "batched":
        return bench_batched(args)
    if args.workload == "kernels":
        return bench_kernels(args)
    if args.workload == "serving":
        return bench_serving(args)
    import torch
    from paper_2412_15122_amd import workloads as W
    from paper_2412_15122_amd.apsp import Graph, kernel_names
    from paper_2412_15122_amd import _native as N

    torch.cuda.set_device(0)
    if args.calibrate_copy:
        src = torch.empty(1 << 28, dtype=torch.int32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    n = args.n
    steps_total = args.warmup + args.steps
    per = args.updates
    counts = {W.ADD: per * 3 // 10, W.REMOVE: per * 2 // 10, W.DECREASE: per // 4, W.INCREASE: per // 4}
    counts[W.INCREASE] = per - counts[W.ADD] - counts[W.REMOVE] - counts[W.DECREASE]
    if args.mix != "all":
        counts = {k: (per if k == args.mix else 0) for k in counts}
    growth = counts[W.ADD] - counts[W.REMOVE]
    cap = n + counts[W.ADD] + 256      # every step starts again from the n-node graph

    t = time.perf_counter()
    adj = W.config3_graph(n)
    log(f"[bench] graph n={n} generated in {time.perf_counter() - t:.1f}s")
    minimax = args.semiring == "minimax"
    base = Graph(adj, undirected=True, capacity=cap, minimax=minimax)
    if args.fallback is not None:
        base.set_fallback(1, args.fallback)
    g = base
    torch.cuda.synchronize()
    log(f"[bench] cold start done ({args.semiring} paths)")
    names = kernel_names()
    kid = {nm: i for i, nm in enumerate(names)}

    # GPU cold blocked Floyd-Warshall at n (median of reps)
    cold_ms = []
    for _ in range(args.cold_reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        g.recompute_cold()
        e1.record()
        torch.cuda.synchronize()
        cold_ms.append(e0.elapsed_time(e1))
    cold_med = float(np.median(cold_ms))
    log(f"[bench] GPU cold FW n={n}: {cold_med:.1f} ms (reps {['%.1f' % c for c in cold_ms]})")

    stream = W.Config3Stream(adj, counts=counts)
    cand_base = W.lightest_edges(adj, 64, True)

    def worst_case_edge():
        """Among the 64 lightest edges of the n-node graph every step starts
        from, the one with the largest |R| * |C| (ties: lowest (u, v))."""
        best, best_key = None, None
        for (u, v, _) in cand_base:
            r, c = base.edge_scope(u, v)
            key = (-(r * c), u, v)
            if best_key is None or key < best_key:
                best, best_key = (u, v), key
        return (best[0], best[1], 20000)

    def stage(block):
        """Upload every add-node weight vector of the block (inputs resident
        in HBM before timing)."""
        vecs = [u.w_out for u in block if u.kind == W.ADD]
        flat = np.concatenate(vecs) if vecs else np.zeros(1, np.int32)
        dev = torch.from_numpy(np.ascontiguousarray(flat, dtype=np.int32)).cuda()
        ptrs, off = [], 0
        for u in block:
            if u.kind == W.ADD:
                ptrs.append(dev.data_ptr() + 4 * off)
                off += u.w_out.size
            else:
                ptrs.append(None)
        return dev, ptrs

    def run_block(g, block, ptrs, events, trace=None):
        for i, u in enumerate(block):
            if u.kind == W.ADD:
                g.add_node_device(ptrs[i], ptrs[i])
            elif u.kind == W.REMOVE:
                g.remove_node(u.u)
            else:
                g.update_edge(u.u, u.v, u.w)
            if events is not None:
                events[i].record()
            if trace is not None and u.kind in (W.REMOVE, W.INCREASE, W.ADD):
                trace.append((u.kind, g.stats()))

    lat_ms = []
    kinds_all = []
    timed_ms = 0.0
    prof_kernel = None
    prof_totals = {}
    alg_bytes_total = 0
    stats_all = []
    # one block of updates, drawn once against the n-node graph; every step
    # restores that graph (a device copy of the cold-started snapshot, outside
    # the timed region) and applies the whole block to it
    worst = worst_case_edge() if counts[W.INCREASE] > 0 else None
    block = stream.next_block(worst=worst)
    dev, ptrs = stage(block)
    live, live_lo, live_hi = n, n, n
    for u in block:
        live += 1 if u.kind == W.ADD else (-1 if u.kind == W.REMOVE else 0)
        live_lo, live_hi = min(live_lo, live), max(live_hi, live)
    # the warm-up steps, the timed steps, then one more untimed step that
    # records an event after every update (per-update latency); the timed
    # steps carry no per-update instrumentation
    for step in range(steps_total + 1):
        timed = args.warmup <= step < steps_total
        latency_step = step == steps_total
        if g is not base:
            g.close()
        g = base.clone()
        torch.cuda.synchronize()
        if step == 0:
            g.profile(-1)          # every kernel: find the dominant one
        elif timed and prof_kernel is not None:
            g.profile(1 << kid[prof_kernel], every=args.prof_every)
        events = [torch.cuda.Event(enable_timing=True) for _ in block] if latency_step else None
        start = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        start.record()
        trace = [] if (args.trace and not timed) else None
        run_block(g, block, ptrs, events, trace)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        if trace:
            for kind in (W.REMOVE, W.INCREASE, W.ADD):
                ss = [st for k, st in trace if k == kind and not st["noop"]]
                if not ss:
                    continue
                keys = ("flagged", "changed", "rows", "rows_changed", "heavy_rows", "sweeps", "full_scans",
                        "rows_relaxed")
                log(f"[bench] trace {kind}: {len(ss)} non-noop; " + ", ".join(
                    f"{k} mean {np.mean([st[k] for st in ss]):.1f} max {max(st[k] for st in ss)}" for k in keys))
        if step == 0:
            tot = {nm: g.profile_read(kid[nm]) for nm in names}
            prof_totals = {nm: v for nm, v in tot.items() if v[0]}
            sweep = {nm: v[1] for nm, v in prof_totals.items() if nm in ("add_relax", "mask_detect")}
            prof_kernel = max(sweep, key=sweep.get) if sweep else None
            g.profile(0)
            log("[bench] kernel totals (step 0): " +
                ", ".join(f"{nm}={v[1]:.1f}ms/{v[0]}" for nm, v in sorted(prof_totals.items(), key=lambda x: -x[1][1])))
        what = "timed" if timed else ("latency, untimed" if latency_step else "warmup")
        log(f"[bench] step {step} ({what}): {1e3 * (t1 - t0):.1f} ms for {len(block)} updates")
        if latency_step:
            prev = start
            for ev in events:
                lat_ms.append(prev.elapsed_time(ev))
                prev = ev
            lat_kinds = [u.kind for u in block]
        if timed:
            timed_ms += 1e3 * (t1 - t0)
            kinds_all += [u.kind for u in block]
            if prof_kernel is not None:
                c, ms = g.profile_read(kid[prof_kernel])
                prof_totals.setdefault("timed", [0, 0.0])
                prof_totals["timed"][0] += c
                prof_totals["timed"][1] += ms
                g.profile(0)
    del dev

    # algorithmic bytes of the dominant kernel over the timed steps: replay the
    # live counts (every add / remove changes n by one; each step starts at n)
    # (only the launches the events timed: 0, every, 2 every, ... of each step)
    removes_bytes = adds_bytes = 0
    launches = {"add_relax": 0, "mask_detect": 0}
    seen = {"add_relax": 0, "mask_detect": 0}
    for t, k in enumerate(kinds_all):
        if t % len(block) == 0:
            live = n
            seen = {"add_relax": 0, "mask_detect": 0}
        if k == W.ADD:
            if seen["add_relax"] % args.prof_every == 0:
                adds_bytes += sweep_bytes("add", live)
                launches["add_relax"] += 1
            seen["add_relax"] += 1
            live += 1
        elif k == W.REMOVE:
            if seen["mask_detect"] % args.prof_every == 0:
                removes_bytes += sweep_bytes("remove", live, count_only=minimax)
                launches["mask_detect"] += 1
            seen["mask_detect"] += 1
            live -= 1
    roofline = None
    if prof_kernel and "timed" in prof_totals and prof_totals["timed"][1] > 0:
        c, ms = prof_totals["timed"]
        if c != launches[prof_kernel]:
            raise RuntimeError(f"{prof_kernel}: {c} timed launches, expected {launches[prof_kernel]}")
        alg = adds_bytes if prof_kernel == "add_relax" else removes_bytes
        achieved = alg / (ms * 1e-3) / 1e9
        tb = None if minimax else traffic_from_profiles(prof_kernel)   # counters were taken on shortest paths
        # the counter runs launch at n = 16384 exactly; this run's launches at
        # the live count of the step: the measured traffic over its
        # algorithmic bytes at that n is the comparable figure
        n_pmc = 16384
        alg_pmc = sweep_bytes("add" if prof_kernel == "add_relax" else "remove", n_pmc)
        roofline = {
            "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": tb,
            "traffic_at_n": n_pmc if tb else None,
            "traffic_vs_algorithmic": round(tb / alg_pmc, 4) if tb else None,
            "kernel": prof_kernel, "launches": c, "timed_every": args.prof_every,
            "avg_launch_ms": round(ms / max(c, 1), 4),
            "algorithmic_bytes_per_launch": round(alg / max(c, 1)),
        }

    if roofline is not None and worst is not None and not minimax:
        roofline["edge_sweep"] = edge_sweep_roofline(base, worst, adj, kid, args.reps_sweep)

    # synchronous single-pair queries on the final graph (host-observed latency)
    qrng = np.random.default_rng(4242)
    live = g.ids()
    q_path, q_nodes, q_cand, q_key = [], [], [], []
    for _ in range(64):
        a, b = (live[int(x)] for x in qrng.integers(0, len(live), size=2))
        t0 = time.perf_counter()
        g.query(a, b)
        t1 = time.perf_counter()
        _, on, key = g.query_nodes(a, b)
        t2 = time.perf_counter()
        q_path.append((t1 - t0) * 1e3)
        q_nodes.append((t2 - t1) * 1e3)
        q_cand.append(len(on))
        q_key.append(len(key))
    query_ms = {"pairs": len(q_path), "path_p50": round(float(np.median(q_path)), 4),
                "nodes_p50": round(float(np.median(q_nodes)), 4),
                "mean_candidates": round(float(np.mean(q_cand)), 2), "mean_key_nodes": round(float(np.mean(q_key)), 2)}
    log(f"[bench] queries: {query_ms}")

    verify = None
    if not args.no_verify:
        # warm result == GPU cold Floyd-Warshall of the final graph
        A_final = g.matrix_device("A")
        D_warm = g.matrix_device("D")
        g2 = Graph(A_final, undirected=True, capacity=A_final.shape[0], minimax=minimax)
        verify = bool(torch.equal(D_warm, g2.matrix_device("D")))
        g2.close()
        del A_final, D_warm
        log(f"[bench] warm == GPU cold on the final graph: {verify}")

    K = args.steps
    ms_per_step = timed_ms / K
    value = per / (ms_per_step * 1e-3)
    lat = np.array(lat_ms)
    by_kind = {}
    for k in (W.ADD, W.REMOVE, W.DECREASE, W.INCREASE):
        sel = np.array([kk == k for kk in lat_kinds])
        if sel.any():
            by_kind[k] = round(float(lat[sel].mean()), 4)
    out = {
        "metric": ("warm-start minimax APSP updates/s (n=16384, 1 GPU)" if minimax
                   else "warm-start APSP updates/s (n=16384, 1 GPU)"),
        "value": round(value, 2),
        "unit": "updates/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "i32",
        "data": "synthetic",
        "config": {
            "workload": (f"undirected complete graph n={n}, symmetric weights U[1,10000], "
                         f"{per} sequential updates per step ({counts[W.ADD]} add / {counts[W.REMOVE]} remove / "
                         f"{counts[W.DECREASE]} decrease / {counts[W.INCREASE]} increase incl. one worst-case increase)"),
            "n": n, "live_nodes_range": [live_lo, live_hi],
            "step": "the n-node graph restored from a snapshot before each step (untimed), then the same block",
            "updates_per_step": per, "parallelism": "none (1 GPU)",
            "paths": args.semiring, "fallback_delta": args.fallback,
        },
        "cold_fw_ms": round(cold_med, 2),
        "cold_updates_per_s": round(1e3 / cold_med, 3),
        "warm_vs_cold_speedup": round(cold_med / (ms_per_step / per), 1),
        "latency_ms": {"p50": round(float(np.percentile(lat, 50)), 4), "p99": round(float(np.percentile(lat, 99)), 4),
                       "mean_by_kind": by_kind,
                       "from": "one extra untimed step of the same block, an event recorded after every update"},
        "query_ms": query_ms,
        "verified_vs_gpu_cold": verify,
        "roofline": roofline,
    }
    g.close()
    base.close()
    del g, base
    torch.cuda.empty_cache()
    legs = [x for x in args.legs.split(",") if x]
    if "batched" in legs and not minimax:
        log("[bench] batched leg: 512 graphs x 8 updates, one persistent launch vs one call per update")
        b = batched_leg(512, 1, 3)
        out["batched"] = {k: b[k] for k in ("metric", "value", "unit", "ms_per_step", "steps", "warmup", "config",
                                            "plain_path", "batched_vs_plain_speedup", "verified_vs_plain",
                                            "roofline")}
        torch.cuda.empty_cache()
    if "serving" in legs and not minimax:
        rates = [float(x) for x in args.leg_rates.split(",")]
        log(f"[bench] serving leg: 64 resident graphs, {args.requests} requests per rate at {rates} req/s")
        sv = serving_leg(64, rates, args.requests, ["lockstep"])
        out["serving"] = {"metric": sv["metric"], "unit": "updates/s", "config": sv["config"],
                          "rates": [{"rate": r["rate"],
                                     "served": {k: r["served"][k] for k in ("updates_per_s", "p50_ms", "p99_ms")},
                                     "plain": {k: r["plain"][k] for k in ("updates_per_s", "p50_ms", "p99_ms")}}
                                    for r in sv["sweep"]]}
        torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        log("[bench] CPU baseline (oracle Floyd-Warshall, sampled)")
        out["cpu_baseline"] = cpu_baseline(adj)
        try:  # context only: a failure here must not cost the benchmark line
            out["cpu_context"] = cpu_context(adj)
        except Exception as e:  # noqa: BLE001
            out["cpu_context"] = {"error": f"{type(e).__name__}: {e}"}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
