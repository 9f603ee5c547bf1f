// Host side of batched updates: item checks against each graph's id map
// (with an undo log, so a rejected batch changes nothing), the grouping of
// items by graph, the upload of the launch records, and the persistent
// launch (direct or replayed from a HIP graph).
#include <algorithm>
#include <cstring>
#include <new>
#include <numeric>
#include <thread>
#include <unordered_set>
#include <vector>

#include "batch_internal.h"
#include "host_graph.h"

using namespace apsp;
using namespace apsp_host;

namespace {

struct BatchLayout {
    size_t graphs, order, items, times, tables, total;
};

BatchLayout batch_layout(int32_t max_graphs, int32_t max_items) {
    BatchLayout L{};
    size_t off = align256(sizeof(BatchHeader));
    L.graphs = off;
    off = align256(off + (size_t)max_graphs * sizeof(BatchGraph));
    L.order = off;
    off = align256(off + (size_t)max_graphs * sizeof(int32_t));
    L.items = off;
    off = align256(off + (size_t)max_items * sizeof(BatchItem));
    L.times = off;
    off = align256(off + (size_t)max_graphs * 2 * sizeof(long long));
    L.tables = off;  // lockstep: per step, add-vector, sweep and recompute chunk prefixes over the graphs, sweep order
    off = align256(off + (size_t)max_items * BATCH_TABLES * ((size_t)max_graphs + 1) * sizeof(int32_t));
    L.total = off;
    return L;
}

struct ExecKey {
    int32_t grid, variant;
    size_t lds;
    bool minimax;
    hipGraph_t graph;
    hipGraphExec_t exec;
};

// One change to a graph's host bookkeeping, undone if a later item fails.
struct Undo {
    apsp_graph *g;
    int32_t op;
    int32_t id, slot, rank, prev_n_slots, prev_max_id;
    bool slot_was_free;
};

// The first item of a graph that failed its checks (t < 0: none).
struct ItemFail {
    int32_t t = -1;
    apsp_status st = APSP_OK;
    const char *what = "";
};

// Host threads that check a batch's items (graphs split between them), from
// this many items on.
constexpr int32_t BATCH_HOST_THREADS = 8;
constexpr int32_t BATCH_HOST_PARALLEL_ITEMS = 512;

void undo_all(std::vector<Undo> &log) {
    for (auto it = log.rbegin(); it != log.rend(); ++it) {
        apsp_graph *g = it->g;
        if (it->op == BOP_ADD) {
            g->live_ids.pop_back();
            g->slot_of_id.erase(it->id);
            g->n_live -= 1;
            g->max_id = it->prev_max_id;
            if (it->slot_was_free) g->free_slots.insert(it->slot);
            g->dg.n_slots = it->prev_n_slots;
        } else if (it->op == BOP_REMOVE) {
            g->live_ids.insert(g->live_ids.begin() + it->rank, it->id);
            g->slot_of_id[it->id] = it->slot;
            g->free_slots.erase(it->slot);
            g->n_live += 1;
            std::swap(g->rank_cur, g->rank_other);
        }
    }
    log.clear();
}

}  // namespace

struct apsp_batch {
    char *ws = nullptr;
    int32_t max_graphs = 0, max_items = 0;
    BatchLayout L{};
    char *stage = nullptr;  // pinned mirror of the workspace
    hipEvent_t staged = nullptr;
    hipEvent_t done = nullptr;
    hipStream_t cap_stream = nullptr;  // launches are recorded here (the null stream cannot be captured)
    std::vector<hipEvent_t> waits;
    bool stage_busy = false;
    int32_t grid = 0, order = 0, variant = 0, use_graph = 0;
    int32_t n_cu = 0;
    int32_t clock_khz = 0;
    long long *times_h = nullptr;  // pinned
    int32_t *err_h = nullptr;      // pinned
    hipStream_t last_stream = nullptr;
    int32_t last_num_graphs = 0, last_steps = 0;
    std::vector<ExecKey> execs;
    // per-run scratch (host)
    std::vector<int32_t> count, begin, fill, active;
    std::vector<int64_t> work;
    std::vector<int32_t> order_items, cursor;  // items grouped by graph; fill cursor
    std::vector<std::vector<Undo>> logs;       // per host thread
};

namespace {

// The batch's graphs share one semiring: minimax picks the apsp::mm build of
// the batched kernels.
apsp_status launch(apsp_batch *b, int32_t n_active, int32_t P_max, bool minimax, hipStream_t s) {
    const bool lockstep = b->variant >= 2;
    int32_t grid = b->grid > 0 ? b->grid : std::max(1, std::min(n_active, 2 * b->n_cu));
    if (lockstep) {
        int32_t cap = 0;
        const hipError_t oc = minimax ? mm::lockstep_grid(P_max, b->variant, &cap) : lockstep_grid(P_max, b->variant, &cap);
        if (!hip_ok(oc, "lockstep occupancy")) return APSP_E_DEVICE;
        grid = b->grid > 0 ? std::min(b->grid, cap) : cap;
    }
    auto *hdr = reinterpret_cast<BatchHeader *>(b->ws);
    auto *graphs = reinterpret_cast<const BatchGraph *>(b->ws + b->L.graphs);
    auto *order = reinterpret_cast<const int32_t *>(b->ws + b->L.order);
    auto *items = reinterpret_cast<const BatchItem *>(b->ws + b->L.items);
    auto *tables = reinterpret_cast<const int32_t *>(b->ws + b->L.tables);
    auto go = [&](hipStream_t st) {
        if (minimax)
            return lockstep ? mm::launch_batch_lockstep(hdr, graphs, items, tables, P_max, grid, b->variant, st)
                            : mm::launch_batch(hdr, graphs, order, items, P_max, grid, b->variant, st);
        return lockstep ? launch_batch_lockstep(hdr, graphs, items, tables, P_max, grid, b->variant, st)
                        : launch_batch(hdr, graphs, order, items, P_max, grid, b->variant, st);
    };
    if (!b->use_graph) {
        hipError_t e = go(s);
        if (e != hipSuccess) return fail(APSP_E_DEVICE, std::string("batched launch: ") + hipGetErrorString(e));
        return APSP_OK;
    }
    const size_t lds = lockstep ? batch_lockstep_lds_bytes(P_max) : batch_lds_bytes(P_max);
    for (auto &x : b->execs) {
        if (x.grid == grid && x.variant == b->variant && x.lds == lds && x.minimax == minimax) {
            if (!hip_ok(hipGraphLaunch(x.exec, s), "graph launch")) return APSP_E_DEVICE;
            return APSP_OK;
        }
    }
    ExecKey k{grid, b->variant, lds, minimax, nullptr, nullptr};
    hipStream_t cs = b->cap_stream;
    if (!hip_ok(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal), "begin capture")) return APSP_E_DEVICE;
    hipError_t e = go(cs);
    hipError_t e2 = hipStreamEndCapture(cs, &k.graph);
    if (e != hipSuccess || e2 != hipSuccess) {
        if (k.graph) (void)hipGraphDestroy(k.graph);
        (void)hipGetLastError();
        return fail(APSP_E_DEVICE, std::string("capturing the batched launch: ") +
                                       hipGetErrorString(e != hipSuccess ? e : e2));
    }
    if (!hip_ok(hipGraphInstantiate(&k.exec, k.graph, nullptr, nullptr, 0), "graph instantiate")) {
        (void)hipGraphDestroy(k.graph);
        return APSP_E_DEVICE;
    }
    b->execs.push_back(k);
    if (!hip_ok(hipGraphLaunch(k.exec, s), "graph launch")) return APSP_E_DEVICE;
    return APSP_OK;
}

// Every host change of the last checks, undone (a later step failed).
void undo_logs(apsp_batch *b) {
    for (auto &l : b->logs) undo_all(l);
}

}  // namespace

extern "C" {

size_t apsp_batch_workspace_bytes(int32_t max_graphs, int32_t max_items) {
    if (max_graphs < 1 || max_items < 1) return 0;
    return batch_layout(max_graphs, max_items).total;
}

apsp_status apsp_batch_create(void *ws_dev, size_t ws_bytes, int32_t max_graphs, int32_t max_items,
                              apsp_batch **out) {
    if (!out) return fail(APSP_E_INVALID, "apsp_batch_create: out is NULL");
    *out = nullptr;
    if (max_graphs < 1 || max_items < 1) return fail(APSP_E_INVALID, "apsp_batch_create: sizes must be >= 1");
    if (!ws_dev || ((uintptr_t)ws_dev & 255) != 0)
        return fail(APSP_E_INVALID, "apsp_batch_create: ws_dev NULL or not 256-byte aligned");
    const BatchLayout L = batch_layout(max_graphs, max_items);
    if (ws_bytes < L.total) return fail(APSP_E_CAPACITY, "apsp_batch_create: ws smaller than apsp_batch_workspace_bytes");
    apsp_batch *b = new (std::nothrow) apsp_batch();
    if (!b) return fail(APSP_E_INVALID, "apsp_batch_create: out of host memory");
    b->ws = (char *)ws_dev;
    b->max_graphs = max_graphs;
    b->max_items = max_items;
    b->L = L;
    int dev = 0;
    if (!hip_ok(hipHostMalloc((void **)&b->stage, L.total, 0), "pinned alloc") ||
        !hip_ok(hipEventCreateWithFlags(&b->staged, hipEventDisableTiming), "event") ||
        !hip_ok(hipEventCreateWithFlags(&b->done, hipEventDisableTiming), "event") ||
        !hip_ok(hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking), "stream") ||
        !hip_ok(hipGetDevice(&dev), "device") ||
        !hip_ok(hipDeviceGetAttribute(&b->n_cu, hipDeviceAttributeMultiprocessorCount, dev), "device attribute") ||
        !hip_ok(hipDeviceGetAttribute(&b->clock_khz, hipDeviceAttributeWallClockRate, dev), "device attribute") ||
        !hip_ok(hipHostMalloc((void **)&b->times_h, (size_t)max_graphs * 2 * sizeof(long long), 0), "pinned alloc") ||
        !hip_ok(hipHostMalloc((void **)&b->err_h, sizeof(int32_t), 0), "pinned alloc") ||
        !hip_ok(configure_batch(), "configuring the batched kernel") ||
        !hip_ok(mm::configure_batch(), "configuring the batched kernel")) {
        apsp_batch_destroy(b);
        return APSP_E_DEVICE;
    }
    std::memset(b->stage, 0, L.total);
    *out = b;
    return APSP_OK;
}

apsp_status apsp_batch_destroy(apsp_batch *b) {
    if (!b) return APSP_OK;
    if (b->staged) (void)hipEventSynchronize(b->staged);
    if (b->done) (void)hipEventSynchronize(b->done);
    for (auto &x : b->execs) {
        if (x.exec) (void)hipGraphExecDestroy(x.exec);
        if (x.graph) (void)hipGraphDestroy(x.graph);
    }
    for (auto e : b->waits) (void)hipEventDestroy(e);
    if (b->staged) (void)hipEventDestroy(b->staged);
    if (b->done) (void)hipEventDestroy(b->done);
    if (b->stage) (void)hipHostFree(b->stage);
    if (b->times_h) (void)hipHostFree(b->times_h);
    if (b->err_h) (void)hipHostFree(b->err_h);
    if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
    delete b;
    return APSP_OK;
}

apsp_status apsp_batch_set_config(apsp_batch *b, int32_t grid, int32_t order, int32_t variant, int32_t use_graph) {
    if (!b) return fail(APSP_E_INVALID, "apsp_batch_set_config: NULL batch");
    if (grid < 0 || order < 0 || order > 1 || variant < 0 || variant > 4 || use_graph < 0 || use_graph > 1)
        return fail(APSP_E_INVALID, "apsp_batch_set_config: value out of range");
    b->grid = grid;
    b->order = order;
    b->variant = variant;
    b->use_graph = use_graph;
    return APSP_OK;
}

apsp_status apsp_batch_run(apsp_batch *b, apsp_graph *const *graphs, int32_t num_graphs,
                           const apsp_batch_item *items, int32_t num_items, void *hip_stream, int32_t *new_ids) {
    if (!b) return fail(APSP_E_INVALID, "apsp_batch_run: NULL batch");
    if (num_graphs < 0 || num_graphs > b->max_graphs) return fail(APSP_E_INVALID, "apsp_batch_run: bad num_graphs");
    if (num_items < 0 || num_items > b->max_items) return fail(APSP_E_INVALID, "apsp_batch_run: bad num_items");
    if ((num_graphs > 0 && !graphs) || (num_items > 0 && !items))
        return fail(APSP_E_INVALID, "apsp_batch_run: NULL array");
    hipStream_t s = (hipStream_t)hip_stream;
    {
        std::unordered_set<const apsp_graph *> seen;
        for (int32_t i = 0; i < num_graphs; ++i) {
            const apsp_graph *g = graphs[i];
            if (!g) return fail(APSP_E_INVALID, "apsp_batch_run: NULL graph " + std::to_string(i));
            if (!seen.insert(g).second) return fail(APSP_E_INVALID, "apsp_batch_run: graph listed twice");
            if (g->detached) return detached_error("apsp_batch_run");
            if (g->minimax != graphs[0]->minimax)
                return fail(APSP_E_INVALID, "apsp_batch_run: the graphs of one batch must share the path kind");
            if (g->cap > BATCH_MAX_CAPACITY)
                return fail(APSP_E_INVALID, "apsp_batch_run: graph capacity above APSP_BATCH_MAX_CAPACITY");
        }
    }
    if (num_items == 0) return APSP_OK;
    // the previous batch's upload must have left the staging buffer
    if (b->stage_busy && !hip_ok(hipEventSynchronize(b->staged), "staging wait")) return APSP_E_DEVICE;
    b->stage_busy = false;
    b->count.assign(num_graphs, 0);
    for (int32_t t = 0; t < num_items; ++t) {
        if (items[t].graph < 0 || items[t].graph >= num_graphs)
            return fail(APSP_E_INVALID, "apsp_batch_run: item " + std::to_string(t) + ": graph index out of range");
        b->count[items[t].graph] += 1;
    }
    b->begin.assign(num_graphs + 1, 0);
    for (int32_t i = 0; i < num_graphs; ++i) b->begin[i + 1] = b->begin[i] + b->count[i];
    b->fill.assign(b->begin.begin(), b->begin.end() - 1);
    b->work.assign(num_graphs, 0);
    auto *bitems = reinterpret_cast<BatchItem *>(b->stage + b->L.items);
    std::vector<int32_t> last_kind(num_graphs, 0), last_n(num_graphs, 0);
    // Each graph's items apply in their order; different graphs' host
    // bookkeeping is independent, so the graphs are split over a few host
    // threads (the per-item checks miss the caches of 512 graphs' id maps).
    // Items grouped by graph, in order:
    b->order_items.resize(num_items);
    b->cursor.assign(b->begin.begin(), b->begin.end() - 1);
    for (int32_t t = 0; t < num_items; ++t) b->order_items[b->cursor[items[t].graph]++] = t;
    // one graph's items; the first failing item stops it (nothing undone here)
    auto run_graph = [&](int32_t gi, std::vector<Undo> &log) -> ItemFail {
        for (int32_t q = b->begin[gi]; q < b->begin[gi + 1]; ++q) {
            const int32_t t = b->order_items[q];
            const apsp_batch_item &x = items[t];
            apsp_graph *g = graphs[x.graph];
            BatchItem bi{};
            bi.rank_src = g->rank_cur;
            if (new_ids) new_ids[t] = -1;
            const bool und = g->kind == APSP_UNDIRECTED;
            if (x.op == APSP_OP_ADD_NODE) {
                if (g->n_live > 0 && (!x.w_out_dev || (!und && !x.w_in_dev)))
                    return ItemFail{t, APSP_E_INVALID, "weight vector is NULL"};
                if (g->max_id >= INT32_MAX - 1) return ItemFail{t, APSP_E_CAPACITY, "the id range is used up"};
                int32_t p;
                bool was_free = false;
                if (!g->free_slots.empty()) {
                    p = *g->free_slots.begin();
                    was_free = true;
                } else if (g->dg.n_slots < g->cap) {
                    p = g->dg.n_slots;
                } else {
                    return ItemFail{t, APSP_E_CAPACITY, "every slot is in use"};
                }
                const int32_t nid = g->max_id + 1;
                log.push_back({g, BOP_ADD, nid, p, 0, g->dg.n_slots, g->max_id, was_free});
                g->dg.n_slots = std::max(g->dg.n_slots, p + 1);
                bi.op = BOP_ADD;
                bi.a = p;
                bi.b = nid;
                bi.c = g->n_live;
                bi.w_out = x.w_out_dev;
                bi.w_in = und ? x.w_out_dev : x.w_in_dev;
                last_kind[x.graph] = UK_ADD;
                last_n[x.graph] = g->n_live;
                g->free_slots.erase(p);
                g->max_id = nid;
                g->live_ids.push_back(nid);
                g->slot_of_id[nid] = p;
                g->n_live += 1;
                if (new_ids) new_ids[t] = nid;
            } else if (x.op == APSP_OP_REMOVE_NODE) {
                int32_t k;
                if (!lookup(g, x.u, &k)) return ItemFail{t, APSP_E_NOT_FOUND, "id is not live"};
                const int32_t r = rank_of(g, x.u);
                log.push_back({g, BOP_REMOVE, x.u, k, r, g->dg.n_slots, g->max_id, false});
                bi.op = BOP_REMOVE;
                bi.a = k;
                bi.b = r;
                bi.c = g->n_live;
                bi.rank_dst = g->rank_other;
                last_kind[x.graph] = UK_REMOVE;
                last_n[x.graph] = g->n_live;
                std::swap(g->rank_cur, g->rank_other);
                g->live_ids.erase(g->live_ids.begin() + r);
                g->slot_of_id.erase(x.u);
                g->free_slots.insert(k);
                g->n_live -= 1;
            } else if (x.op == APSP_OP_UPDATE_EDGE) {
                if (x.w < 0 || (uint32_t)x.w > INF) return ItemFail{t, APSP_E_INVALID, "weight outside [0, APSP_INF]"};
                if (x.u == x.v) return ItemFail{t, APSP_E_INVALID, "u == v"};
                int32_t su, sv;
                if (!lookup(g, x.u, &su) || !lookup(g, x.v, &sv)) return ItemFail{t, APSP_E_NOT_FOUND, "id is not live"};
                bi.op = BOP_EDGE;
                bi.a = su;
                bi.b = sv;
                bi.c = g->dg.widest ? widest_xf(x.w) : x.w;
                last_kind[x.graph] = -1;
                last_n[x.graph] = g->n_live;
            } else if (x.op == APSP_OP_QUERY) {
                int32_t si, sj;
                if (!lookup(g, x.u, &si) || !lookup(g, x.v, &sj)) return ItemFail{t, APSP_E_NOT_FOUND, "id is not live"};
                if (!x.out_dev || x.out_cap < 3 + g->n_live) return ItemFail{t, APSP_E_CAPACITY, "query output too short"};
                bi.op = BOP_QUERY;
                bi.a = si;
                bi.b = sj;
                bi.out = x.out_dev;
            } else {
                return ItemFail{t, APSP_E_INVALID, "unknown op"};
            }
            bi.n_slots = g->dg.n_slots;
            b->work[x.graph] += (int64_t)bi.n_slots * bi.n_slots;
            bitems[b->fill[x.graph]++] = bi;
        }
        return ItemFail{};
    };
    const int32_t nthreads = num_items >= BATCH_HOST_PARALLEL_ITEMS
                                 ? std::max(1, std::min<int32_t>(BATCH_HOST_THREADS, num_graphs))
                                 : 1;
    b->logs.resize(nthreads);
    std::vector<ItemFail> fails(nthreads);
    // contiguous ranges of graphs with about equal item counts
    auto run_range = [&](int32_t w) {
        b->logs[w].clear();
        const int64_t lo = (int64_t)num_items * w / nthreads, hi = (int64_t)num_items * (w + 1) / nthreads;
        for (int32_t gi = 0; gi < num_graphs; ++gi) {
            if (b->begin[gi] < lo || b->begin[gi] >= hi || b->count[gi] == 0) continue;
            const ItemFail f = run_graph(gi, b->logs[w]);
            if (f.t >= 0) {
                fails[w] = f;
                return;
            }
        }
    };
    if (nthreads == 1) {
        run_range(0);
    } else {
        std::vector<std::thread> pool;
        pool.reserve(nthreads - 1);
        for (int32_t w = 1; w < nthreads; ++w) pool.emplace_back(run_range, w);
        run_range(0);
        for (auto &th : pool) th.join();
    }
    const ItemFail *first = nullptr;
    for (const ItemFail &f : fails)
        if (f.t >= 0 && (!first || f.t < first->t)) first = &f;
    if (first) {
        undo_logs(b);
        return fail(first->st, "apsp_batch_run: item " + std::to_string(first->t) + ": " + first->what);
    }
    // launch records: graphs with items, most work first unless asked otherwise
    auto *hdr = reinterpret_cast<BatchHeader *>(b->stage);
    auto *bgraphs = reinterpret_cast<BatchGraph *>(b->stage + b->L.graphs);
    auto *order = reinterpret_cast<int32_t *>(b->stage + b->L.order);
    b->active.clear();
    int32_t P_max = 1;
    for (int32_t i = 0; i < num_graphs; ++i) {
        if (b->count[i] == 0) continue;
        apsp_graph *g = graphs[i];
        BatchGraph &bg = bgraphs[b->active.size()];
        bg.g = g->dg;
        bg.wo = wo(g);
        bg.wi = wi(g);
        bg.vout = vout(g);
        bg.vin = vin(g);
        bg.colu = colu(g);
        bg.colv = colv(g);
        bg.rowu = rowu(g);
        bg.rowv = rowv(g);
        bg.plist = g->plist;
        bg.plist_cnt = g->plist_cnt;
        bg.plist_beta = g->plist_beta;
        bg.scratch = g->fscratch;
        bg.qscratch = g->qscratch;
        bg.queue = g->nin_queue;
        bg.flag_bits = g->flag_bits;
        bg.row_bits = g->row_bits;
        bg.heavy_rows = g->heavy_rows;
        bg.item_begin = b->begin[i];
        bg.item_end = b->begin[i + 1];
        bg.index = i;
        P_max = std::max(P_max, g->P);
        b->active.push_back(i);
    }
    const int32_t n_active = (int32_t)b->active.size();
    std::vector<int32_t> ord(n_active);
    std::iota(ord.begin(), ord.end(), 0);
    if (b->order == 0)
        std::stable_sort(ord.begin(), ord.end(),
                         [&](int32_t x, int32_t y) { return b->work[b->active[x]] > b->work[b->active[y]]; });
    std::copy(ord.begin(), ord.end(), order);
    hdr->num_graphs = n_active;
    hdr->counter = 0;
    hdr->times = reinterpret_cast<long long *>(b->ws + b->L.times);
    hdr->p_max = P_max;
    hdr->steps = 0;
    size_t table_words = 0;
    if (b->variant >= 2) {
        // lockstep: step s applies item s of every graph; per step, the chunk
        // prefixes of the add-vector phase (additions), the sweep phase
        // (every kind but a query) and the recompute phase (removals and
        // edge updates), and the order of the sweep and recompute prefixes:
        // additions and removals (which always sweep) by falling byte count,
        // then the edge updates (which sweep only when phase A finds the edge
        // matters)
        int32_t steps = 0;
        for (int32_t i : b->active) steps = std::max(steps, b->count[i]);
        auto *tab = reinterpret_cast<int32_t *>(b->stage + b->L.tables);
        const int32_t G1 = n_active + 1;
        std::vector<int64_t> sweep_key(n_active);
        std::vector<int32_t> sweep_cb(n_active), sweep_cc(n_active);
        for (int32_t st = 0; st < steps; ++st) {
            int32_t *ta = tab + (size_t)st * BATCH_TABLES * G1, *tb = ta + G1, *tc = tb + G1, *td = tc + G1;
            ta[0] = tb[0] = tc[0] = 0;
            for (int32_t ai = 0; ai < n_active; ++ai) {
                const int32_t i = b->active[ai];
                int32_t ca = 0, cb = 0, cc = 0;
                int64_t key = 0;
                if (st < b->count[i]) {
                    const BatchItem &bi = bitems[b->begin[i] + st];
                    const int32_t rpc = batch_rows_per_chunk(bi.n_slots);
                    // with staged sweeps the sweep chunks compute a directed
                    // add's new column themselves (batch.hip, sweep_chunk)
                    if (bi.op == BOP_ADD)
                        ca = lockstep_stages_sweeps(P_max) ? add_out_chunks(bi.n_slots)
                                                           : add_vec_chunks(bi.n_slots, graphs[i]->kind == APSP_UNDIRECTED);
                    if (bi.op != BOP_QUERY) cb = (bi.n_slots + rpc - 1) / rpc;
                    if (bi.op == BOP_REMOVE || bi.op == BOP_EDGE)
                        cc = (bi.n_slots + BATCH_RECOMPUTE_ROWS - 1) / BATCH_RECOMPUTE_ROWS;
                    if (bi.op == BOP_ADD || bi.op == BOP_REMOVE) key = (int64_t)bi.n_slots * bi.n_slots;
                }
                ta[ai + 1] = ta[ai] + ca;
                sweep_cb[ai] = cb;
                sweep_cc[ai] = cc;
                sweep_key[ai] = key;
                td[ai] = ai;
            }
            td[n_active] = 0;
            std::stable_sort(td, td + n_active, [&](int32_t x, int32_t y) { return sweep_key[x] > sweep_key[y]; });
            for (int32_t k = 0; k < n_active; ++k) {
                tb[k + 1] = tb[k] + sweep_cb[td[k]];
                tc[k + 1] = tc[k] + sweep_cc[td[k]];
            }
        }
        hdr->steps = steps;
        b->last_steps = steps;
        table_words = (size_t)steps * BATCH_TABLES * G1;
    }
    // order the batch after earlier work of each graph on its own stream
    std::vector<hipStream_t> others;
    for (int32_t i : b->active)
        if (graphs[i]->stream != s && std::find(others.begin(), others.end(), graphs[i]->stream) == others.end())
            others.push_back(graphs[i]->stream);
    while (b->waits.size() < others.size()) {
        hipEvent_t e;
        if (!hip_ok(hipEventCreateWithFlags(&e, hipEventDisableTiming), "event")) return undo_logs(b), APSP_E_DEVICE;
        b->waits.push_back(e);
    }
    for (size_t q = 0; q < others.size(); ++q)
        if (!hip_ok(hipEventRecord(b->waits[q], others[q]), "event record") ||
            !hip_ok(hipStreamWaitEvent(s, b->waits[q], 0), "stream wait"))
            return undo_logs(b), APSP_E_DEVICE;
    const size_t bytes = b->L.items + (size_t)num_items * sizeof(BatchItem);
    if (!hip_ok(hipMemcpyAsync(b->ws, b->stage, bytes, hipMemcpyHostToDevice, s), "batch upload") ||
        (table_words && !hip_ok(hipMemcpyAsync(b->ws + b->L.tables, b->stage + b->L.tables,
                                               table_words * sizeof(int32_t), hipMemcpyHostToDevice, s),
                                "batch upload")) ||
        !hip_ok(hipEventRecord(b->staged, s), "event record"))
        return undo_logs(b), APSP_E_DEVICE;
    b->stage_busy = true;
    apsp_status st = launch(b, n_active, P_max, num_graphs > 0 && graphs[0]->minimax, s);
    if (st) return undo_logs(b), st;
    // later single calls on a graph's own stream run after the batch
    if (!others.empty()) {
        if (!hip_ok(hipEventRecord(b->done, s), "event record")) return APSP_E_DEVICE;
        for (hipStream_t o : others)
            if (!hip_ok(hipStreamWaitEvent(o, b->done, 0), "stream wait")) return APSP_E_DEVICE;
    }
    b->last_stream = s;
    b->last_num_graphs = num_graphs;
    for (int32_t i : b->active) {
        apsp_graph *g = graphs[i];
        if (last_kind[i] != 0) {
            g->last_kind = last_kind[i];
            g->stats_pending = 0;  // the batch sums its own statistics
            g->last_n_before = last_n[i];
            g->last_fallback = 0;
        }
    }
    for (auto &l : b->logs) l.clear();
    return APSP_OK;
}

apsp_status apsp_batch_graph_times(apsp_batch *b, double *start_us, double *end_us, int32_t num_graphs) {
    if (!b || !start_us || !end_us) return fail(APSP_E_INVALID, "apsp_batch_graph_times: NULL argument");
    if (num_graphs != b->last_num_graphs)
        return fail(APSP_E_INVALID, "apsp_batch_graph_times: num_graphs differs from the last run");
    if (num_graphs == 0) return APSP_OK;
    const size_t bytes = (size_t)num_graphs * 2 * sizeof(long long);
    if (!hip_ok(hipMemcpyAsync(b->times_h, b->ws + b->L.times, bytes, hipMemcpyDeviceToHost, b->last_stream), "copy") ||
        !hip_ok(hipStreamSynchronize(b->last_stream), "stream sync"))
        return APSP_E_DEVICE;
    std::vector<char> ran(num_graphs, 0);
    for (int32_t i : b->active) ran[i] = 1;
    long long t0 = 0;
    bool first = true;
    for (int32_t i = 0; i < num_graphs; ++i)
        if (ran[i] && (first || b->times_h[2 * i] < t0)) {
            t0 = b->times_h[2 * i];
            first = false;
        }
    const double us_per_tick = 1e3 / (double)std::max(1, b->clock_khz);
    for (int32_t i = 0; i < num_graphs; ++i) {
        start_us[i] = ran[i] ? (double)(b->times_h[2 * i] - t0) * us_per_tick : -1.0;
        end_us[i] = ran[i] ? (double)(b->times_h[2 * i + 1] - t0) * us_per_tick : -1.0;
    }
    return APSP_OK;
}

apsp_status apsp_batch_status(apsp_batch *b) {
    if (!b) return fail(APSP_E_INVALID, "apsp_batch_status: NULL batch");
    if (b->last_num_graphs == 0) return APSP_OK;
    auto *hdr = reinterpret_cast<BatchHeader *>(b->ws);
    if (!hip_ok(hipMemcpyAsync(b->err_h, &hdr->err, sizeof(int32_t), hipMemcpyDeviceToHost, b->last_stream), "copy") ||
        !hip_ok(hipStreamSynchronize(b->last_stream), "stream sync"))
        return APSP_E_DEVICE;
    if (b->variant >= 2 && *b->err_h)
        return fail(APSP_E_DEVICE, "apsp_batch_status: a grid barrier of the lockstep launch timed out; the "
                                   "batch's graphs are in an undefined state");
    return APSP_OK;
}

apsp_status apsp_batch_phase_times(apsp_batch *b, double *us, int32_t cap, int32_t *count) {
    if (!b || !count || (cap > 0 && !us)) return fail(APSP_E_INVALID, "apsp_batch_phase_times: bad argument");
    *count = 0;
    if (b->variant < 2 || b->last_num_graphs == 0) return APSP_OK;
    auto *hdr = reinterpret_cast<BatchHeader *>(b->ws);
    std::vector<long long> ts(BATCH_PHASE_STAMPS + 2);
    long long *stamps = ts.data();
    if (!hip_ok(hipMemcpyAsync(stamps, hdr->phase_ts, BATCH_PHASE_STAMPS * sizeof(long long), hipMemcpyDeviceToHost,
                               b->last_stream),
                "copy") ||
        !hip_ok(hipMemcpyAsync(b->times_h, b->ws + b->L.times, 2 * sizeof(long long), hipMemcpyDeviceToHost,
                               b->last_stream),
                "copy") ||
        !hip_ok(hipStreamSynchronize(b->last_stream), "stream sync"))
        return APSP_E_DEVICE;
    std::vector<long long> work(BATCH_PHASE_STAMPS);
    if (!hip_ok(hipMemcpy(work.data(), hdr->work_ts, BATCH_PHASE_STAMPS * sizeof(long long), hipMemcpyDeviceToHost),
                "copy"))
        return APSP_E_DEVICE;
    const int32_t n = std::min(cap, std::min(3 * b->last_steps, BATCH_PHASE_STAMPS));
    const double us_per_tick = 1e3 / (double)std::max(1, b->clock_khz);
    long long t0 = b->times_h[0];  // start of the first graph
    for (int32_t k = 0; k < n; ++k) us[k] = (double)(stamps[k] - t0) * us_per_tick;
    // diagnostics: the latest end of recompute work of step s goes after the
    // phase ends, when there is room
    for (int32_t s2 = 0; s2 < b->last_steps && n + s2 < cap && s2 < BATCH_PHASE_STAMPS; ++s2)
        us[n + s2] = work[s2] ? (double)(work[s2] - t0) * us_per_tick : 0.0;
    *count = std::min(cap, n + std::min(b->last_steps, BATCH_PHASE_STAMPS));
    return APSP_OK;
}

}  // extern "C"
