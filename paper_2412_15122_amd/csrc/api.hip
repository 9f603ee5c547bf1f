// Host side of the C ABI: argument checks, the id <-> slot map, buffer
// carving, and the order in which each update enqueues its kernels.
#include <algorithm>
#include <cstdio>
#include <cstring>
#include <new>
#include <set>
#include <string>
#include <unordered_map>
#include <vector>

#include "apsp_internal.h"

using namespace apsp;
// The launcher of g's semiring: namespace apsp for shortest paths, apsp::mm
// for minimax paths (the same kernel sources, compiled once per semiring).
#define SR(g, fn) ((g)->minimax ? &mm::fn : &fn)

#include "host_graph.h"
#include "msf.h"

using namespace apsp_host;

thread_local std::string apsp_host::g_err;

namespace apsp {
void Prof::begin(int32_t kid) {
    auto *p = static_cast<apsp_host::ProfImpl *>(impl);
    // launches 0, every, 2 every, ... of each enabled kernel are timed
    if (!on || !p || !((p->mask >> kid) & 1) || p->seen[kid]++ % p->every != 0) {
        if (p) p->cur_kid = -1;
        return;
    }
    hipEvent_t e = p->take();
    if (!e) return;
    (void)hipEventRecord(e, p->stream);
    p->cur_kid = kid;
    p->cur_a = e;
}
void Prof::end() {
    auto *p = static_cast<apsp_host::ProfImpl *>(impl);
    if (!on || !p || p->cur_kid < 0) return;
    hipEvent_t e = p->take();
    if (!e) return;
    (void)hipEventRecord(e, p->stream);
    p->recs.push_back({p->cur_kid, p->cur_a, e});
    p->cur_kid = -1;
}
}  // namespace apsp

namespace {

// The statistics an edge update left as partials (see update_edge_with),
// summed into the control block.
apsp_status flush_stats(apsp_graph *g) {
    if (!g->stats_pending) return APSP_OK;
    launch_edge_stats(g->dg, g->partials, g->stats_pending, g->stream);
    g->stats_pending = 0;
    return check_launch("edge update statistics");
}

apsp_status read_ctl(apsp_graph *g) {
    if (!hip_ok(hipMemcpyAsync(g->ctl_h, g->dg.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, g->stream), "read ctl"))
        return APSP_E_DEVICE;
    if (!hip_ok(hipStreamSynchronize(g->stream), "stream sync")) return APSP_E_DEVICE;
    return APSP_OK;
}

// D := cold Floyd-Warshall of the current adjacency over the used slots.
apsp_status run_cold(apsp_graph *g) {
    const int32_t n = g->dg.n_slots;
    g->prof.begin(KID_MISC);
    launch_copy_square(g->dg.D, g->dg.A, g->dg.ld, n, g->stream);
    g->prof.end();
    apsp_status st = check_launch("cold start copy");
    if (st) return st;
    if (const char *bad = SR(g, launch_fw)(g->dg, n, g->stream, &g->prof))
        return fail(APSP_E_DEVICE, std::string("Floyd-Warshall launch failed: ") + bad);
    return APSP_OK;
}

// Algorithm 5's switch, after the mask has been detected (Phi and |F| are in
// the control block): 1 when cold Floyd-Warshall should replace the masked
// recompute.  Only the cost policy reads the counts back (synchronous).
apsp_status decide_fallback(apsp_graph *g, const FusedArgs *fa, int32_t n_before, int32_t *fallback) {
    *fallback = 0;
    if (g->policy == APSP_FALLBACK_ALWAYS) {
        *fallback = 1;
        return APSP_OK;
    }
    if (g->policy != APSP_FALLBACK_COST) return APSP_OK;
    launch_count_flag_rows(g->dg, *fa, g->stream);
    apsp_status st = read_ctl(g);
    if (st) return st;
    const double cost = n_before > 1 ? (double)g->ctl_h->rows / (double)(n_before - 1) : 0.0;
    *fallback = cost > g->delta;
    launch_fill(&g->dg.ctl->rows, 1, 0, g->stream);  // the recompute counts Phi again
    return check_launch("cost decision");
}

// The spanning forest, its certificate and the pieces of T - k (or of T - e
// for a raised edge eu-ev of old weight ew), read back into g->qbuf_h.
// Boruvka needs at most about log2(n) rounds but usually far fewer: a first
// try runs 10 (the rounds after convergence are launches that do nothing),
// and only a forest still growing after them is built again with all.
apsp_status build_forest(apsp_graph *g, const MsfWork &w, int32_t k, int32_t eu, int32_t ev, int32_t ew,
                         int32_t n_before, const char *who) {
    int32_t rounds = 2;
    while ((1 << (rounds - 2)) < std::max(n_before, 2)) ++rounds;
    const int32_t first = std::min<int32_t>(rounds, 10);
    for (int32_t r : {first, rounds}) {
        launch_msf_forest(g->dg, w, k, eu, ev, ew, r, g->stream);
        if (apsp_status st = check_launch(who)) return st;
        if (!hip_ok(hipMemcpyAsync(g->qbuf_h, w.info, 8 * sizeof(int32_t), hipMemcpyDeviceToHost, g->stream),
                    "forest read") ||
            !hip_ok(hipStreamSynchronize(g->stream), "stream sync"))
            return APSP_E_DEVICE;
        if (g->qbuf_h[MI_ACTIVE] == 0 || r == rounds) break;
    }
    return APSP_OK;
}

// Removal of slot k from an undirected minimax graph through its minimum
// spanning forest (msf.hip): the forest over the light index, its
// certificate and the pieces of T - k, one read-back, then -- when the
// certificate holds -- the mask's counts and the new entries of the pairs
// across pieces.  *used is false when the certificate or a size limit
// rejects the forest (nothing written: the caller runs the mask route);
// *fallback is 1 when Algorithm 5's cost test picks cold Floyd-Warshall
// (no entry written either).
apsp_status remove_by_forest(apsp_graph *g, int32_t k, int32_t n_before, bool *used, int32_t *fallback) {
    *used = false;
    *fallback = 0;
    if (msf_configure() != hipSuccess) {
        (void)hipGetLastError();
        return APSP_OK;
    }
    DevGraph &d = g->dg;
    hipStream_t s = g->stream;
    const MsfWork w = msf_work(g->fscratch, g->P);
    if (w.ints > (int64_t)FUSED_GRID * 2 * g->P) return APSP_OK;  // the heavy-row scratch holds it (P >= 128)
    apsp_status st = build_forest(g, w, k, -1, -1, 0, n_before, "apsp_remove_node: spanning forest");
    if (st) return st;
    const int32_t *info = g->qbuf_h;
    if (info[MI_ACTIVE] != 0 || info[MI_FAIL] != 0) return APSP_OK;
    FusedArgs fa{};
    fa.mode = FUSED_REMOVE;
    fa.k = k;
    fa.col1 = colu(g);
    fa.row1 = rowu(g);
    g->prof.begin(KID_MASK);
    mm::launch_mask_count(d, fa, s);
    g->prof.end();
    *used = true;
    if (g->policy == APSP_FALLBACK_COST) {
        if ((st = read_ctl(g))) return st;
        const double cost = n_before > 1 ? (double)g->ctl_h->rows / (double)(n_before - 1) : 0.0;
        if (cost > g->delta) {
            *fallback = 1;
            return check_launch("apsp_remove_node: mask counts");
        }
    }
    g->prof.begin(KID_FUSED);
    launch_msf_update(d, w, info[MI_SMALL], s);
    g->prof.end();
    return check_launch("apsp_remove_node: spanning-forest update");
}

// A tight increase of edge (su, sv) from w_old on an undirected minimax graph
// through its minimum spanning forest (msf.hip), after k_edge_begin has
// written the new weight: the forest of the graph before the change, its
// certificate and the two pieces of T - e, one read-back, then -- when the
// certificate holds -- the mask's counts and the new entries of the pairs
// across the pieces (none when e is not in T).  *used and *fallback as in
// remove_by_forest.
apsp_status increase_by_forest(apsp_graph *g, int32_t su, int32_t sv, int32_t w_old, int32_t n_before, bool *used,
                               int32_t *fallback, const FusedArgs &fa) {
    *used = false;
    *fallback = 0;
    if (msf_configure() != hipSuccess) {
        (void)hipGetLastError();
        return APSP_OK;
    }
    DevGraph &d = g->dg;
    hipStream_t s = g->stream;
    const MsfWork w = msf_work(g->fscratch, g->P);
    if (w.ints > (int64_t)FUSED_GRID * 2 * g->P) return APSP_OK;
    apsp_status st = build_forest(g, w, -1, su, sv, w_old, n_before, "apsp_update_edge: spanning forest");
    if (st) return st;
    const int32_t *info = g->qbuf_h;
    if (info[MI_ACTIVE] != 0 || info[MI_FAIL] != 0) return APSP_OK;
    const int32_t pieces = info[MI_D], small = info[MI_SMALL];
    g->prof.begin(KID_MASK);
    mm::launch_mask_count(d, fa, s);
    g->prof.end();
    *used = true;
    if (g->policy == APSP_FALLBACK_COST) {
        if ((st = read_ctl(g))) return st;
        const double cost = n_before > 1 ? (double)g->ctl_h->rows / (double)(n_before - 1) : 0.0;
        if (cost > g->delta) {
            *fallback = 1;
            return check_launch("apsp_update_edge: mask counts");
        }
    }
    if (pieces == 2) {
        g->prof.begin(KID_FUSED);
        launch_msf_update(d, w, small, s);
        g->prof.end();
    }
    return check_launch("apsp_update_edge: spanning-forest update");
}

// A handle over the caller's buffer: pinned host mirrors and the carving of
// dev_buf by make_layout; nothing is enqueued.
apsp_status make_handle(int32_t capacity, int32_t kind, void *dev_buf, hipStream_t stream, apsp_graph **out) {
    const Layout L = make_layout(capacity, kind);
    apsp_graph *g = new (std::nothrow) apsp_graph();
    if (!g) return fail(APSP_E_INVALID, "out of host memory");
    g->cap = capacity;
    g->P = padded(capacity);
    g->kind = kind;
    g->stream = stream;
    g->base = (char *)dev_buf;
    if (!hip_ok(hipHostMalloc((void **)&g->ctl_h, sizeof(Ctl), 0), "pinned alloc") ||
        !hip_ok(hipHostMalloc((void **)&g->qbuf_h, (size_t)(2 * g->P + 8) * 4, 0), "pinned alloc")) {
        apsp_graph_destroy(g);
        return APSP_E_DEVICE;
    }
    char *b = g->base;
    DevGraph &d = g->dg;
    d.D = (int32_t *)(b + L.D);
    d.A = (int32_t *)(b + L.A);
    d.AT = kind == APSP_DIRECTED ? (int32_t *)(b + L.AT) : nullptr;
    d.nin = (int2 *)(b + L.nin);
    d.nin_cnt = (int32_t *)(b + L.nin_cnt);
    d.nin_beta = (int32_t *)(b + L.nin_beta);
    d.id_of_slot = (int32_t *)(b + L.id_of_slot);
    d.ctl = (Ctl *)(b + L.ctl);
    d.ld = g->P;
    d.P = g->P;
    d.n_slots = 0;
    d.undirected = kind == APSP_UNDIRECTED;
    d.lim = NIN_L;
    for (int v = 0; v < NVEC; ++v) g->vec[v] = (int32_t *)(b + L.vec) + (size_t)v * g->P;
    g->plist = (int2 *)(b + L.plist);
    g->plist_cnt = (int32_t *)(b + L.plist + NIN_L * sizeof(int2));
    g->plist_beta = g->plist_cnt + 1;
    g->rank_cur = (int32_t *)(b + L.rank_a);
    g->rank_other = (int32_t *)(b + L.rank_b);
    g->qbuf = (int32_t *)(b + L.qbuf);
    g->qscratch = (int32_t *)(b + L.qscratch);
    g->fscratch = (int32_t *)(b + L.fscratch);
    g->nin_queue = (int32_t *)(b + L.nin_queue);
    g->heavy_rows = (int32_t *)(b + L.heavy_rows);
    g->heavy_epoch = (int32_t *)(b + L.heavy_epoch);
    g->flag_bits = (uint32_t *)(b + L.flag_bits);
    g->row_bits = (uint32_t *)(b + L.row_bits);
    g->marks = (uint8_t *)(b + L.marks);
    g->partials = (int32_t *)(b + L.partials);
    g->prof_impl.stream = g->stream;
    g->prof.impl = &g->prof_impl;

    *out = g;
    return APSP_OK;
}

FusedArgs fused_args(apsp_graph *g, int32_t mode) {
    FusedArgs fa{};
    fa.mode = mode;
    fa.k = -1;
    fa.scratch = g->fscratch;
    fa.heavy_rows = g->heavy_rows;
    fa.heavy_epoch = g->heavy_epoch;
    fa.flag_bits = g->flag_bits;
    fa.row_bits = g->row_bits;
    fa.marks = g->marks;
    fa.mark_pitch = mark_pitch(g->P);
    fa.partials = g->partials;
    fa.epoch = ++g->epoch;
    return fa;
}

// Every buffer of a new handle in its initial state: no edges, no
// distances (INF), no ids, empty index lists, clear flags and counters.
apsp_status init_buffers(apsp_graph *g) {
    DevGraph &d = g->dg;
    hipStream_t s = g->stream;
    const int64_t PP = (int64_t)g->P * g->P;
    launch_fill(d.D, PP, (int32_t)INF, s);
    launch_fill(d.A, PP, (int32_t)INF, s);
    if (d.AT) launch_fill(d.AT, PP, (int32_t)INF, s);
    launch_fill(d.id_of_slot, g->P, -1, s);
    launch_fill(d.nin_cnt, g->P, 0, s);
    launch_fill(d.nin_beta, g->P, (int32_t)INF, s);
    launch_fill(g->heavy_epoch, g->P, 0, s);
    launch_fill((int32_t *)g->row_bits, (g->P + 31) / 32, 0, s);
    launch_fill((int32_t *)g->flag_bits, (int64_t)g->P * ((g->P + 31) / 32), 0, s);
    launch_fill((int32_t *)d.ctl, sizeof(Ctl) / 4, 0, s);
    return check_launch("initial fill");
}

// The part of a new graph that precedes its distance matrix: argument
// checks, the handle, every buffer in its initial state, the adjacency (and
// its transpose) loaded, slots 0..n-1 in use.  Messages start with `who`.
apsp_status new_graph(const char *who, const int32_t *adj_dev, int32_t n, int64_t adj_ld, int32_t kind,
                      int32_t capacity, void *dev_buf, size_t dev_buf_bytes, void *hip_stream, apsp_graph **out,
                      apsp_graph **made) {
    const std::string w(who);
    if (!out) return fail(APSP_E_INVALID, w + ": out is NULL");
    *out = nullptr;
    const int32_t dir = kind & ~(int32_t)(APSP_MINIMAX | APSP_WIDEST);
    if (dir != APSP_DIRECTED && dir != APSP_UNDIRECTED) return fail(APSP_E_INVALID, w + ": bad kind");
    if ((kind & APSP_MINIMAX) && (kind & APSP_WIDEST))
        return fail(APSP_E_INVALID, w + ": APSP_MINIMAX and APSP_WIDEST exclude each other");
    if (capacity < 1 || capacity > APSP_MAX_CAPACITY)
        return fail(APSP_E_INVALID, w + ": capacity must be in [1, APSP_MAX_CAPACITY]");
    if (n < 0 || n > capacity) return fail(APSP_E_INVALID, w + ": n must be in [0, capacity]");
    if (n > 0 && (!adj_dev || adj_ld < n)) return fail(APSP_E_INVALID, w + ": bad adjacency pointer or ld");
    if (!dev_buf) return fail(APSP_E_INVALID, w + ": dev_buf is NULL");
    if (((uintptr_t)dev_buf & 255) != 0) return fail(APSP_E_INVALID, w + ": dev_buf not 256-byte aligned");
    const Layout L = make_layout(capacity, dir);
    if (dev_buf_bytes < L.total) return fail(APSP_E_CAPACITY, w + ": dev_buf smaller than apsp_required_bytes");

    apsp_graph *g = nullptr;
    apsp_status st0 = make_handle(capacity, dir, dev_buf, (hipStream_t)hip_stream, &g);
    if (st0) return st0;
    // widest paths are minimax paths over transformed weights (widest_xf)
    g->minimax = (kind & (APSP_MINIMAX | APSP_WIDEST)) != 0;
    DevGraph &d = g->dg;
    d.widest = (kind & APSP_WIDEST) != 0;
    hipError_t ce = configure_kernels();
    if (ce == hipSuccess) ce = mm::configure_kernels();
    if (hipError_t e = ce; e != hipSuccess) {
        apsp_graph_destroy(g);
        return fail(APSP_E_DEVICE, std::string("configuring kernels: ") + hipGetErrorString(e));
    }
    hipStream_t s = g->stream;
    apsp_status st = init_buffers(g);
    if (st) {
        apsp_graph_destroy(g);
        return st;
    }
    launch_load_adj(d, adj_dev, adj_ld, n, s);
    if (d.AT) launch_transpose(d.A, d.AT, d.ld, n, s);
    d.n_slots = n;
    launch_iota(d.id_of_slot, n, s);
    launch_iota(g->rank_cur, n, s);
    if ((st = check_launch("cold start load"))) {
        apsp_graph_destroy(g);
        return st;
    }
    *made = g;
    return APSP_OK;
}

// The part that follows D: the light in-edge index and the host's id map
// (ids[r] for slot r, or 0..n-1 when ids is NULL).
apsp_status finish_graph(apsp_graph *g, int32_t n, const int32_t *ids) {
    launch_nin_build(g->dg, 0, n, 0, g->stream);
    apsp_status st = check_launch("index build");
    if (st) return st;
    g->n_live = n;
    g->live_ids.resize(n);
    for (int32_t i = 0; i < n; ++i) {
        g->live_ids[i] = ids ? ids[i] : i;
        g->slot_of_id[g->live_ids[i]] = i;
    }
    g->max_id = n > 0 ? g->live_ids[n - 1] : -1;
    return APSP_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------

// The edge update over given working memory (the public entry points below
// pass the graph's own or the library's static array).
apsp_status apsp_host::check_edge_args(apsp_graph *g, const char *who, int32_t u, int32_t v, int32_t w, int32_t *su,
                                       int32_t *sv) {
    if (!g) return fail(APSP_E_INVALID, std::string(who) + ": NULL graph");
    if (g->detached) return detached_error(who);
    if (w < 0 || (uint32_t)w > INF) return fail(APSP_E_INVALID, std::string(who) + ": weight outside [0, APSP_INF]");
    if (u == v) return fail(APSP_E_INVALID, std::string(who) + ": u == v");
    if (!lookup(g, u, su) || !lookup(g, v, sv)) return fail(APSP_E_NOT_FOUND, std::string(who) + ": id is not live");
    return APSP_OK;
}

apsp_status apsp_host::update_edge_with(apsp_graph *g, const char *who, int32_t u, int32_t v, int32_t w,
                                        const EdgeScratch &sc) {
    int32_t su, sv;
    if (apsp_status bad = check_edge_args(g, who, u, v, w, &su, &sv)) return bad;
    if (g->dg.widest) w = widest_xf(w);  // a capacity, stored as its transform
    hipStream_t s = g->stream;
    DevGraph &d = g->dg;
    const int32_t n_before = g->n_live;
    g->prof.begin(KID_EDGE_BEGIN);
    launch_edge_begin(d, su, sv, w, sc.colu, sc.colv, sc.rowu, sc.rowv, sc.marks, s);
    g->prof.end();
    FusedArgs fa{};
    fa.mode = FUSED_INCREASE;
    fa.k = -1;
    fa.scratch = sc.fscratch;
    fa.heavy_rows = sc.heavy_rows;
    fa.heavy_epoch = sc.heavy_epoch;
    fa.flag_bits = sc.flag_bits;
    fa.row_bits = sc.row_bits;
    fa.marks = sc.marks;
    fa.mark_pitch = mark_pitch(g->P);
    fa.partials = sc.partials;
    fa.epoch = sc.epoch;
    fa.col1 = sc.colu;
    fa.col2 = sc.colv;
    fa.row1 = sc.rowv;
    fa.row2 = sc.rowu;
    apsp_status st;
    // undirected minimax graphs: a tight increase takes the spanning-forest
    // route when its certificate holds (it works in the graph's own memory,
    // so not for the no-allocation entry point); the device's decision is
    // read back first
    if (g->minimax && g->kind == APSP_UNDIRECTED && g->P <= MSF_MAX_PITCH && sc.lazy_stats &&
        g->policy != APSP_FALLBACK_ALWAYS) {
        if ((st = read_ctl(g))) return st;
        if (g->ctl_h->edge_mode == EDGE_INCREASE) {
            bool forest = false;
            int32_t fb = 0;
            if ((st = increase_by_forest(g, su, sv, g->ctl_h->w_old, n_before, &forest, &fb, fa))) return st;
            if (forest) {
                if (fb && (st = run_cold(g))) return st;
                if ((st = check_launch(who))) return st;
                g->stats_pending = 0;
                g->last_n_before = n_before;
                g->last_fallback = fb;
                g->last_kind = -1;
                g->last_route = 1;
                return APSP_OK;
            }
        }
    }
    g->prof.begin(KID_EDGE_SWEEP);
    SR(g, launch_edge_sweep)(d, fa, w, s);
    g->prof.end();
    int32_t fallback = 0;
    if (g->policy != APSP_FALLBACK_NEVER) {
        if ((st = read_ctl(g))) return st;
        if (g->ctl_h->edge_mode == EDGE_INCREASE && (st = decide_fallback(g, &fa, n_before, &fallback))) return st;
    }
    g->prof.begin(KID_FUSED);
    const int32_t rblocks = SR(g, launch_mask_recompute)(d, fa, fallback, s);
    g->prof.end();
    if (fallback && (st = run_cold(g))) return st;
    // the recompute's statistics stay as per-work-group partials in the
    // graph's own memory until they are read; memory shared with other calls
    // is summed at once
    if (sc.lazy_stats) {
        g->stats_pending = rblocks;
    } else {
        launch_edge_stats(d, sc.partials, rblocks, s);
        g->stats_pending = 0;
    }
    if ((st = check_launch(who))) return st;
    g->last_n_before = n_before;
    g->last_fallback = fallback;
    g->last_kind = -1;  // the device picked the path; apsp_last_stats reads it back
    g->last_route = 0;
    return APSP_OK;
}

extern "C" {

int32_t apsp_abi_version(void) { return APSP_ABI_VERSION; }

const char *apsp_last_error(void) { return g_err.c_str(); }

int32_t apsp_kernel_count(void) { return KID_COUNT; }

const char *apsp_kernel_name(int32_t k) {
    static const char *names[KID_COUNT] = {
        "fw_pivot", "fw_panel", "fw_tiles", "nin_build", "nin_update", "add_out", "add_in", "add_relax",
        "add_place", "gather", "mask_recompute", "tombstone", "edge_begin", "edge_sweep", "query", "misc",
        "mask_detect"};
    if (k < 0 || k >= KID_COUNT) return "";
    return names[k];
}

size_t apsp_required_bytes(int32_t capacity, int32_t kind) {
    if (capacity < 1 || capacity > APSP_MAX_CAPACITY) return 0;
    const int32_t dir = kind & ~(int32_t)(APSP_MINIMAX | APSP_WIDEST);
    if (dir != APSP_DIRECTED && dir != APSP_UNDIRECTED) return 0;
    if ((kind & APSP_MINIMAX) && (kind & APSP_WIDEST)) return 0;
    return make_layout(capacity, dir).total;
}

apsp_status apsp_cold(const int32_t *adj_dev, int32_t n, int64_t adj_ld, int32_t kind, int32_t capacity,
                      void *dev_buf, size_t dev_buf_bytes, void *hip_stream, apsp_graph **out) {
    apsp_graph *g = nullptr;
    apsp_status st = new_graph("apsp_cold", adj_dev, n, adj_ld, kind, capacity, dev_buf, dev_buf_bytes, hip_stream,
                               out, &g);
    if (st) return st;
    if ((st = run_cold(g)) || (st = finish_graph(g, n, nullptr))) {
        apsp_graph_destroy(g);
        return st;
    }
    *out = g;
    return APSP_OK;
}

apsp_status apsp_import(const int32_t *adj_dev, int64_t adj_ld, const int32_t *apsp_dev, int64_t apsp_ld,
                        int32_t n, const int32_t *ids, int32_t next_id, int32_t kind, int32_t capacity,
                        void *dev_buf, size_t dev_buf_bytes, void *hip_stream, int32_t verify, apsp_graph **out) {
    if (out) *out = nullptr;
    if (verify != APSP_IMPORT_TRUSTED && verify != APSP_IMPORT_EXACT)
        return fail(APSP_E_INVALID, "apsp_import: verify must be APSP_IMPORT_TRUSTED or APSP_IMPORT_EXACT");
    if (n > 0 && (!apsp_dev || apsp_ld < n)) return fail(APSP_E_INVALID, "apsp_import: bad matrix pointer or ld");
    if (ids) {
        for (int32_t i = 0; i < n; ++i)
            if (ids[i] < 0 || ids[i] == INT32_MAX || (i > 0 && ids[i] <= ids[i - 1]))
                return fail(APSP_E_INVALID, "apsp_import: ids must be non-negative and strictly ascending");
    }
    const int32_t top = n == 0 ? -1 : ids ? ids[n - 1] : n - 1;
    if (next_id != -1 && (next_id <= top || next_id == INT32_MAX))
        return fail(APSP_E_INVALID, "apsp_import: next_id must exceed every id and be below INT32_MAX (or be -1)");
    apsp_graph *g = nullptr;
    apsp_status st = new_graph("apsp_import", adj_dev, n, adj_ld, kind, capacity, dev_buf, dev_buf_bytes, hip_stream,
                               out, &g);
    if (st) return st;
    hipStream_t s = g->stream;
    int32_t *bad = g->qscratch;  // free until the first query
    launch_fill(bad, 1, 0, s);
    launch_import_d(g->dg, apsp_dev, apsp_ld, n, bad, s);
    if (verify == APSP_IMPORT_EXACT) {
        st = run_cold(g);
        if (!st) launch_count_diff(g->dg.D, g->dg.ld, apsp_dev, apsp_ld, n, bad, g->dg.widest, s);
    }
    if (!st && ids && n > 0 &&
        !hip_ok(hipMemcpyAsync(g->dg.id_of_slot, ids, (size_t)n * 4, hipMemcpyHostToDevice, s), "ids copy"))
        st = APSP_E_DEVICE;
    if (!st) st = check_launch("apsp_import");
    if (!st && (!hip_ok(hipMemcpyAsync(g->qbuf_h, bad, 4, hipMemcpyDeviceToHost, s), "check copy") ||
                !hip_ok(hipStreamSynchronize(s), "stream sync")))
        st = APSP_E_DEVICE;
    if (!st && g->qbuf_h[0] != 0)
        st = fail(APSP_E_INVALID, "apsp_import: " + std::to_string(g->qbuf_h[0]) +
                                      (verify == APSP_IMPORT_EXACT
                                           ? " entries fail the checks or differ from the cold recompute"
                                           : " entries fail the checks of a distance matrix"));
    if (!st) st = finish_graph(g, n, ids);
    if (!st && next_id != -1) g->max_id = next_id - 1;
    if (st) {
        apsp_graph_destroy(g);
        return st;
    }
    *out = g;
    return APSP_OK;
}

apsp_status apsp_recompute_cold(apsp_graph *g) {
    if (!g) return fail(APSP_E_INVALID, "apsp_recompute_cold: NULL graph");
    if (g->detached) return detached_error("apsp_recompute_cold");
    return run_cold(g);
}

apsp_status apsp_graph_destroy(apsp_graph *g) {
    if (!g) return APSP_OK;
    (void)hipStreamSynchronize(g->stream);
    if (g->ctl_h) (void)hipHostFree(g->ctl_h);
    if (g->qbuf_h) (void)hipHostFree(g->qbuf_h);
    delete g;
    return APSP_OK;
}

apsp_status apsp_graph_clone(apsp_graph *g, void *dev_buf, size_t dev_buf_bytes, void *hip_stream,
                             apsp_graph **out) {
    if (!out) return fail(APSP_E_INVALID, "apsp_graph_clone: out is NULL");
    *out = nullptr;
    if (!g) return fail(APSP_E_INVALID, "apsp_graph_clone: NULL graph");
    if (g->detached) return detached_error("apsp_graph_clone");
    if (!dev_buf) return fail(APSP_E_INVALID, "apsp_graph_clone: dev_buf is NULL");
    if (((uintptr_t)dev_buf & 255) != 0) return fail(APSP_E_INVALID, "apsp_graph_clone: dev_buf not 256-byte aligned");
    const Layout L = make_layout(g->cap, g->kind);
    if (dev_buf_bytes < L.total) return fail(APSP_E_CAPACITY, "apsp_graph_clone: dev_buf smaller than apsp_required_bytes");
    if ((char *)dev_buf < g->base + L.total && g->base < (char *)dev_buf + L.total)
        return fail(APSP_E_INVALID, "apsp_graph_clone: dev_buf overlaps the source graph");
    apsp_status st = flush_stats(g);  // the copy carries the summed statistics
    if (st) return st;
    apsp_graph *c = nullptr;
    st = make_handle(g->cap, g->kind, dev_buf, (hipStream_t)hip_stream, &c);
    if (st) return st;
    hipEvent_t ev = nullptr;
    bool ok = hip_ok(hipEventCreateWithFlags(&ev, hipEventDisableTiming), "event") &&
              hip_ok(hipEventRecord(ev, g->stream), "event record") &&
              hip_ok(hipStreamWaitEvent(c->stream, ev, 0), "stream wait") &&
              hip_ok(hipMemcpyAsync(c->base, g->base, L.total, hipMemcpyDeviceToDevice, c->stream), "clone copy") &&
              // g's later calls must not overwrite the source while it is copied
              (c->stream == g->stream || (hip_ok(hipEventRecord(ev, c->stream), "event record") &&
                                          hip_ok(hipStreamWaitEvent(g->stream, ev, 0), "stream wait")));
    if (ev) (void)hipEventDestroy(ev);
    if (!ok) {
        apsp_graph_destroy(c);
        return APSP_E_DEVICE;
    }
    const int64_t ro = (char *)g->rank_cur - g->base;
    c->rank_cur = (int32_t *)(c->base + ro);
    c->rank_other = (int32_t *)(c->base + ((char *)g->rank_other - g->base));
    c->dg.n_slots = g->dg.n_slots;
    c->dg.lim = g->dg.lim;
    c->dg.widest = g->dg.widest;
    c->epoch = g->epoch;
    c->n_live = g->n_live;
    c->max_id = g->max_id;
    c->live_ids = g->live_ids;
    c->slot_of_id = g->slot_of_id;
    c->free_slots = g->free_slots;
    c->policy = g->policy;
    c->delta = g->delta;
    c->last_kind = g->last_kind;
    c->minimax = g->minimax;
    c->last_n_before = g->last_n_before;
    c->last_fallback = g->last_fallback;
    *out = c;
    return APSP_OK;
}

apsp_status apsp_grow(apsp_graph *g, int32_t capacity, void *dev_buf, size_t dev_buf_bytes, void *hip_stream,
                      apsp_graph **out) {
    if (!out) return fail(APSP_E_INVALID, "apsp_grow: out is NULL");
    *out = nullptr;
    if (!g) return fail(APSP_E_INVALID, "apsp_grow: NULL graph");
    if (g->detached) return detached_error("apsp_grow");
    if (capacity < g->dg.n_slots || capacity < 1 || capacity > APSP_MAX_CAPACITY)
        return fail(APSP_E_INVALID, "apsp_grow: capacity must be in [slots in use, APSP_MAX_CAPACITY]");
    if (!dev_buf || ((uintptr_t)dev_buf & 255) != 0)
        return fail(APSP_E_INVALID, "apsp_grow: dev_buf NULL or not 256-byte aligned");
    const Layout L = make_layout(capacity, g->kind);
    if (dev_buf_bytes < L.total) return fail(APSP_E_CAPACITY, "apsp_grow: dev_buf smaller than apsp_required_bytes");
    const size_t src_total = make_layout(g->cap, g->kind).total;
    if ((char *)dev_buf < g->base + src_total && g->base < (char *)dev_buf + L.total)
        return fail(APSP_E_INVALID, "apsp_grow: dev_buf overlaps the source graph");
    if (apsp_status fs = flush_stats(g)) return fs;  // the copy carries the summed statistics
    apsp_graph *c = nullptr;
    apsp_status st = make_handle(capacity, g->kind, dev_buf, (hipStream_t)hip_stream, &c);
    if (st) return st;
    c->minimax = g->minimax;
    hipStream_t cs = c->stream;
    const int32_t ns = g->dg.n_slots;
    const DevGraph &gd = g->dg;
    DevGraph &cd = c->dg;
    hipEvent_t ev = nullptr;
    bool ok = hip_ok(hipEventCreateWithFlags(&ev, hipEventDisableTiming), "event") &&
              hip_ok(hipEventRecord(ev, g->stream), "event record") &&
              hip_ok(hipStreamWaitEvent(cs, ev, 0), "stream wait") && init_buffers(c) == APSP_OK;
    // slot s keeps its place: rows and columns [0, ns) of each matrix move to
    // the wider pitch, the per-slot tables and the rank table are copied
    auto copy2d = [&](int32_t *dst, const int32_t *src) {
        return ns == 0 || hip_ok(hipMemcpy2DAsync(dst, (size_t)c->P * 4, src, (size_t)g->P * 4, (size_t)ns * 4, ns,
                                                  hipMemcpyDeviceToDevice, cs),
                                 "grow copy");
    };
    auto copy1d = [&](void *dst, const void *src, size_t bytes) {
        return bytes == 0 || hip_ok(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, cs), "grow copy");
    };
    ok = ok && copy2d(cd.D, gd.D) && copy2d(cd.A, gd.A) && (!gd.AT || copy2d(cd.AT, gd.AT)) &&
         copy1d(cd.nin, gd.nin, (size_t)ns * NIN_L * sizeof(int2)) && copy1d(cd.nin_cnt, gd.nin_cnt, (size_t)ns * 4) &&
         copy1d(cd.nin_beta, gd.nin_beta, (size_t)ns * 4) && copy1d(cd.id_of_slot, gd.id_of_slot, (size_t)ns * 4) &&
         copy1d(c->rank_cur, g->rank_cur, (size_t)g->n_live * 4) && copy1d(cd.ctl, gd.ctl, sizeof(Ctl)) &&
         // g's later calls must not overwrite the source while it is copied
         (cs == g->stream ||
          (hip_ok(hipEventRecord(ev, cs), "event record") && hip_ok(hipStreamWaitEvent(g->stream, ev, 0), "stream wait")));
    if (ev) (void)hipEventDestroy(ev);
    if (!ok) {
        apsp_graph_destroy(c);
        return APSP_E_DEVICE;
    }
    cd.n_slots = ns;
    cd.lim = gd.lim;
    cd.widest = gd.widest;
    c->epoch = g->epoch;
    c->n_live = g->n_live;
    c->max_id = g->max_id;
    c->live_ids = g->live_ids;
    c->slot_of_id = g->slot_of_id;
    c->free_slots = g->free_slots;
    c->policy = g->policy;
    c->delta = g->delta;
    c->last_kind = g->last_kind;
    c->last_n_before = g->last_n_before;
    c->last_fallback = g->last_fallback;
    *out = c;
    return APSP_OK;
}

apsp_status apsp_graph_relocate(apsp_graph *g, void *dev_buf, size_t dev_buf_bytes) {
    if (!g) return fail(APSP_E_INVALID, "apsp_graph_relocate: NULL graph");
    if (!dev_buf || ((uintptr_t)dev_buf & 255) != 0)
        return fail(APSP_E_INVALID, "apsp_graph_relocate: dev_buf NULL or not 256-byte aligned");
    const Layout L = make_layout(g->cap, g->kind);
    if (dev_buf_bytes < L.total) return fail(APSP_E_CAPACITY, "apsp_graph_relocate: dev_buf smaller than apsp_required_bytes");
    apsp_graph *t = nullptr;
    apsp_status st = make_handle(g->cap, g->kind, dev_buf, g->stream, &t);
    if (st) return st;
    const int64_t rc = (char *)g->rank_cur - g->base, ro = (char *)g->rank_other - g->base;
    const int32_t n_slots = g->dg.n_slots, lim = g->dg.lim, widest = g->dg.widest;
    g->base = t->base;
    g->dg = t->dg;
    g->dg.n_slots = n_slots;
    g->dg.lim = lim;
    g->dg.widest = widest;
    for (int v = 0; v < NVEC; ++v) g->vec[v] = t->vec[v];
    g->plist = t->plist;
    g->plist_cnt = t->plist_cnt;
    g->plist_beta = t->plist_beta;
    g->rank_cur = (int32_t *)(g->base + rc);
    g->rank_other = (int32_t *)(g->base + ro);
    g->qbuf = t->qbuf;
    g->qscratch = t->qscratch;
    g->fscratch = t->fscratch;
    g->nin_queue = t->nin_queue;
    g->heavy_rows = t->heavy_rows;
    g->heavy_epoch = t->heavy_epoch;
    g->flag_bits = t->flag_bits;
    g->row_bits = t->row_bits;
    g->marks = t->marks;
    g->partials = t->partials;
    g->detached = 0;
    apsp_graph_destroy(t);
    return APSP_OK;
}

apsp_status apsp_graph_detach(apsp_graph *g) {
    if (!g) return fail(APSP_E_INVALID, "apsp_graph_detach: NULL graph");
    if (!g->detached)
        if (apsp_status st = flush_stats(g)) return st;
    if (!hip_ok(hipStreamSynchronize(g->stream), "stream sync")) return APSP_E_DEVICE;
    g->detached = 1;
    return APSP_OK;
}

apsp_status apsp_set_stream(apsp_graph *g, void *hip_stream) {
    if (!g) return fail(APSP_E_INVALID, "apsp_set_stream: NULL graph");
    g->stream = (hipStream_t)hip_stream;
    g->prof_impl.stream = g->stream;
    return APSP_OK;
}

apsp_status apsp_set_fallback(apsp_graph *g, int32_t policy, double delta) {
    if (!g) return fail(APSP_E_INVALID, "apsp_set_fallback: NULL graph");
    if (policy < APSP_FALLBACK_NEVER || policy > APSP_FALLBACK_ALWAYS)
        return fail(APSP_E_INVALID, "apsp_set_fallback: bad policy");
    if (!(delta >= 0.0)) return fail(APSP_E_INVALID, "apsp_set_fallback: delta must be >= 0");
    g->policy = policy;
    g->delta = delta;
    return APSP_OK;
}

apsp_status apsp_set_index_limit(apsp_graph *g, int32_t limit) {
    if (!g) return fail(APSP_E_INVALID, "apsp_set_index_limit: NULL graph");
    if (limit < 1 || limit > NIN_L) return fail(APSP_E_INVALID, "apsp_set_index_limit: limit must be in [1, 64]");
    g->dg.lim = limit;
    return APSP_OK;
}

apsp_status apsp_add_node(apsp_graph *g, const int32_t *w_out_dev, const int32_t *w_in_dev, int32_t *new_id) {
    if (!g || !new_id) return fail(APSP_E_INVALID, "apsp_add_node: NULL argument");
    if (g->detached) return detached_error("apsp_add_node");
    const bool und = g->kind == APSP_UNDIRECTED;
    if (g->n_live > 0 && (!w_out_dev || (!und && !w_in_dev)))
        return fail(APSP_E_INVALID, "apsp_add_node: weight vector is NULL");
    // ids stay below INT32_MAX, as apsp_import requires of the ids it takes
    if (g->max_id >= INT32_MAX - 1) return fail(APSP_E_CAPACITY, "apsp_add_node: the id range is used up");
    int32_t p;
    if (!g->free_slots.empty()) p = *g->free_slots.begin();
    else if (g->dg.n_slots < g->cap) p = g->dg.n_slots;
    else return fail(APSP_E_CAPACITY, "apsp_add_node: every slot is in use");
    const int32_t nid = g->max_id + 1;
    hipStream_t s = g->stream;
    DevGraph &d = g->dg;
    const int32_t n_before = g->n_live;
    d.n_slots = std::max(d.n_slots, p + 1);
    launch_scatter_weights(d, w_out_dev, w_in_dev, g->rank_cur, n_before, wo(g), und ? wo(g) : wi(g), s);
    int32_t *wi_s = und ? wo(g) : wi(g);
    int2 *pin = d.nin + (int64_t)p * NIN_L;
    g->prof.begin(KID_NIN_BUILD);
    launch_select_vec(wi_s, d.n_slots, p, pin, d.nin_cnt + p, d.nin_beta + p, s);
    if (!und) launch_select_vec(wo(g), d.n_slots, p, g->plist, g->plist_cnt, g->plist_beta, s);
    g->prof.end();
    const int2 *ol = und ? pin : g->plist;
    const int32_t *oc = und ? d.nin_cnt + p : g->plist_cnt;
    const int32_t *ob = und ? d.nin_beta + p : g->plist_beta;
    g->prof.begin(KID_ADD_OUT);
    SR(g, launch_add_out)(d, ol, oc, ob, wo(g), vout(g), s);
    g->prof.end();
    int32_t *in = vout(g);
    if (!und) {
        g->prof.begin(KID_ADD_IN);
        SR(g, launch_add_in)(d, p, wi_s, vin(g), s);
        g->prof.end();
        in = vin(g);
    }
    g->prof.begin(KID_ADD_RELAX);
    SR(g, launch_add_relax)(d, in, vout(g), s);
    g->prof.end();
    g->prof.begin(KID_ADD_PLACE);
    launch_add_finish(d, p, nid, n_before, g->rank_cur, in, vout(g), wo(g), wi_s, s);
    g->prof.end();
    apsp_status st = check_launch("apsp_add_node");
    if (st) return st;
    g->free_slots.erase(p);
    g->max_id = nid;
    g->live_ids.push_back(nid);
    g->slot_of_id[nid] = p;
    g->n_live += 1;
    g->last_kind = UK_ADD;
    g->stats_pending = 0;
    g->last_n_before = n_before;
    g->last_fallback = 0;
    *new_id = nid;
    return APSP_OK;
}

apsp_status apsp_remove_node(apsp_graph *g, int32_t id) {
    if (!g) return fail(APSP_E_INVALID, "apsp_remove_node: NULL graph");
    if (g->detached) return detached_error("apsp_remove_node");
    int32_t k;
    if (!lookup(g, id, &k)) return fail(APSP_E_NOT_FOUND, "apsp_remove_node: id is not live");
    const int32_t r = rank_of(g, id);
    hipStream_t s = g->stream;
    DevGraph &d = g->dg;
    const int32_t n_before = g->n_live;
    g->prof.begin(KID_GATHER);
    launch_remove_begin(d, k, colu(g), rowu(g), g->marks, s);
    g->prof.end();
    int32_t fallback = 0;
    apsp_status st;
    // undirected minimax graphs: the spanning-forest route when its
    // certificate holds (exact, and it writes only the changed pairs)
    bool forest = false;
    if (g->minimax && g->kind == APSP_UNDIRECTED && g->P <= MSF_MAX_PITCH && g->policy != APSP_FALLBACK_ALWAYS &&
        (st = remove_by_forest(g, k, n_before, &forest, &fallback)))
        return st;
    int32_t rblocks = 0;
    if (!forest) {
        FusedArgs fa = fused_args(g, FUSED_REMOVE);
        fa.k = k;
        fa.col1 = colu(g);
        fa.row1 = rowu(g);
        g->prof.begin(KID_MASK);
        SR(g, launch_mask_detect)(d, fa, s);
        g->prof.end();
        if ((st = decide_fallback(g, &fa, n_before, &fallback))) return st;
        g->prof.begin(KID_FUSED);
        rblocks = SR(g, launch_mask_recompute)(d, fa, fallback, s);
        g->prof.end();
    }
    g->prof.begin(KID_TOMBSTONE);
    launch_remove_finish(d, k, g->nin_queue, g->rank_cur, g->rank_other, r, n_before, g->partials, rblocks, s);
    g->prof.end();
    if (fallback) {
        if ((st = run_cold(g))) return st;
    }
    g->prof.begin(KID_NIN_BUILD);
    launch_nin_rebuild_queue(d, g->nin_queue, s);
    g->prof.end();
    if ((st = check_launch("apsp_remove_node"))) return st;
    std::swap(g->rank_cur, g->rank_other);
    g->live_ids.erase(g->live_ids.begin() + r);
    g->slot_of_id.erase(id);
    g->free_slots.insert(k);
    g->n_live -= 1;
    g->last_kind = UK_REMOVE;
    g->stats_pending = 0;
    g->last_n_before = n_before;
    g->last_fallback = fallback;
    g->last_route = forest ? 1 : 0;
    return APSP_OK;
}

apsp_status apsp_update_edge(apsp_graph *g, int32_t u, int32_t v, int32_t w) {
    int32_t su, sv;
    if (apsp_status bad = check_edge_args(g, "apsp_update_edge", u, v, w, &su, &sv)) return bad;
    // the graph's own working memory, carved from its buffer
    EdgeScratch sc{};
    sc.colu = colu(g);
    sc.colv = colv(g);
    sc.rowu = rowu(g);
    sc.rowv = rowv(g);
    sc.fscratch = g->fscratch;
    sc.heavy_rows = g->heavy_rows;
    sc.heavy_epoch = g->heavy_epoch;
    sc.flag_bits = g->flag_bits;
    sc.row_bits = g->row_bits;
    sc.marks = g->marks;
    sc.partials = g->partials;
    sc.lazy_stats = true;
    sc.epoch = ++g->epoch;
    return update_edge_with(g, "apsp_update_edge", u, v, w, sc);
}

apsp_status apsp_query(apsp_graph *g, int32_t i, int32_t j, int32_t *dist, int32_t *path_ids, int32_t path_cap,
                       int32_t *path_len) {
    if (!g || !dist || !path_len) return fail(APSP_E_INVALID, "apsp_query: NULL argument");
    if (g->detached) return detached_error("apsp_query");
    if (path_cap < 0 || (path_cap > 0 && !path_ids)) return fail(APSP_E_INVALID, "apsp_query: bad path buffer");
    int32_t si, sj;
    if (!lookup(g, i, &si) || !lookup(g, j, &sj)) return fail(APSP_E_NOT_FOUND, "apsp_query: id is not live");
    hipStream_t s = g->stream;
    g->prof.begin(KID_QUERY);
    if (g->minimax) {
        if (const char *bad = mm::launch_query_bottleneck(g->dg, si, sj, g->qbuf, g->qscratch, g->qbuf_h, s)) {
            g->prof.end();
            return fail(APSP_E_DEVICE, std::string("apsp_query: ") + bad);
        }
    } else {
        launch_query(g->dg, si, sj, g->qbuf, g->qscratch, s);
    }
    g->prof.end();
    apsp_status st = check_launch("apsp_query");
    if (st) return st;
    const size_t words = 3 + (size_t)std::min(g->n_live, std::max(path_cap, 1));
    if (!hip_ok(hipMemcpyAsync(g->qbuf_h, g->qbuf, words * 4, hipMemcpyDeviceToHost, s), "query copy") ||
        !hip_ok(hipStreamSynchronize(s), "query sync"))
        return APSP_E_DEVICE;
    if (g->qbuf_h[2] != 0) return fail(APSP_E_DEVICE, "apsp_query: no shortest path found on the device");
    *dist = g->dg.widest ? widest_xf(g->qbuf_h[0]) : g->qbuf_h[0];
    *path_len = g->qbuf_h[1];
    if (*path_len > path_cap) return fail(APSP_E_CAPACITY, "apsp_query: path_cap too small");
    for (int32_t t = 0; t < *path_len; ++t) path_ids[t] = g->qbuf_h[3 + t];
    return APSP_OK;
}

apsp_status apsp_query_nodes(apsp_graph *g, int32_t i, int32_t j, int32_t *dist, int32_t *on_ids, int32_t on_cap,
                             int32_t *on_len, int32_t *key_ids, int32_t key_cap, int32_t *key_len) {
    if (!g || !dist || !on_len || !key_len) return fail(APSP_E_INVALID, "apsp_query_nodes: NULL argument");
    if (g->detached) return detached_error("apsp_query_nodes");
    if (on_cap < 0 || (on_cap > 0 && !on_ids) || key_cap < 0 || (key_cap > 0 && !key_ids))
        return fail(APSP_E_INVALID, "apsp_query_nodes: bad output buffer");
    int32_t si, sj;
    if (!lookup(g, i, &si) || !lookup(g, j, &sj)) return fail(APSP_E_NOT_FOUND, "apsp_query_nodes: id is not live");
    hipStream_t s = g->stream;
    const int32_t n = g->n_live;
    // output: 4 + 2 n ints at the start of the heavy-pass scratch; the
    // per-work-group search space after it (the scratch is idle between updates)
    int32_t *out = g->fscratch;
    int32_t *bfs = g->fscratch + (((size_t)2 * g->P + 8 + 63) & ~(size_t)63);
    g->prof.begin(KID_QUERY);
    if (g->minimax) {
        // output, then n_slots marks; the candidate arrays and the path after them
        int32_t *work = g->fscratch + (((size_t)3 * g->P + 72 + 63) & ~(size_t)63);
        if (const char *bad = mm::launch_query_nodes_bottleneck(g->dg, si, sj, g->rank_cur, n, out, g->qscratch, work,
                                                                g->qbuf_h, s)) {
            g->prof.end();
            return fail(APSP_E_DEVICE, std::string("apsp_query_nodes: ") + bad);
        }
    } else {
        launch_query_nodes(g->dg, si, sj, g->rank_cur, n, out, g->qscratch, bfs, s);
    }
    g->prof.end();
    apsp_status st = check_launch("apsp_query_nodes");
    if (st) return st;
    if (!hip_ok(hipMemcpyAsync(g->qbuf_h, out, (size_t)(4 + 2 * n) * 4, hipMemcpyDeviceToHost, s), "query copy") ||
        !hip_ok(hipStreamSynchronize(s), "query sync"))
        return APSP_E_DEVICE;
    *dist = g->dg.widest ? widest_xf(g->qbuf_h[0]) : g->qbuf_h[0];
    *on_len = g->qbuf_h[1];
    *key_len = g->qbuf_h[2];
    if (*on_len > on_cap || *key_len > key_cap) return fail(APSP_E_CAPACITY, "apsp_query_nodes: buffer too small");
    std::copy(g->qbuf_h + 4, g->qbuf_h + 4 + *on_len, on_ids);
    std::copy(g->qbuf_h + 4 + n, g->qbuf_h + 4 + n + *key_len, key_ids);
    return APSP_OK;
}

apsp_status apsp_query_paths(apsp_graph *g, int32_t i, int32_t j, int32_t *dist, int32_t *ids, int64_t ids_cap,
                             int64_t *ids_len, int32_t *offsets, int32_t offsets_cap, int32_t *npaths) {
    if (!g || !dist || !ids_len || !npaths) return fail(APSP_E_INVALID, "apsp_query_paths: NULL argument");
    if (g->detached) return detached_error("apsp_query_paths");
    if (ids_cap < 0 || (ids_cap > 0 && !ids) || offsets_cap < 0 || (offsets_cap > 0 && !offsets))
        return fail(APSP_E_INVALID, "apsp_query_paths: bad output buffer");
    int32_t si, sj;
    if (!lookup(g, i, &si) || !lookup(g, j, &sj)) return fail(APSP_E_NOT_FOUND, "apsp_query_paths: id is not live");
    const int32_t n = g->n_live;
    // the nodes on some shortest path (the candidates), and the query's own path
    std::vector<int32_t> on(std::max(n, 1)), key(std::max(n, 1)), first(std::max(n, 1));
    int32_t d = 0, on_len = 0, key_len = 0, first_len = 0;
    apsp_status st = apsp_query_nodes(g, i, j, &d, on.data(), n, &on_len, key.data(), n, &key_len);
    if (st) return st;
    *dist = d;
    if (on_len == 0) {  // unreachable
        *npaths = 0;
        *ids_len = 0;
        if (offsets_cap >= 1) offsets[0] = 0;
        return offsets_cap >= 1 ? APSP_OK : fail(APSP_E_CAPACITY, "apsp_query_paths: offsets_cap too small");
    }
    if ((st = apsp_query(g, i, j, &d, first.data(), n, &first_len))) return st;
    first.resize(first_len);
    std::set<int32_t> on_first(first.begin(), first.end());
    std::vector<int32_t> cand;  // slots of the candidates off the first path, ascending id
    for (int32_t x = 0; x < on_len; ++x) {
        const int32_t t = on[x];
        if (t == i || t == j || on_first.count(t)) continue;
        int32_t st_ = 0;
        lookup(g, t, &st_);
        cand.push_back(st_);
    }
    std::vector<std::vector<int32_t>> paths{first};
    std::set<std::vector<int32_t>> seen{first};
    // chunks of candidates, one work-group each, over the heavy-row scratch
    // (idle between updates): candidate slots, 4 P words of query scratch
    // per work-group, two query outputs of P + 3 words per work-group
    const int64_t P = g->P, room = (int64_t)FUSED_GRID * 2 * P - 256;
    const int32_t chunk = (int32_t)std::max<int64_t>(1, std::min<int64_t>(128, room / (4 * P + 2 * (P + 3))));
    int32_t *cslots = g->fscratch;
    int32_t *qsc = g->fscratch + 256;
    int32_t *qout = qsc + (int64_t)chunk * 4 * P;
    hipStream_t s = g->stream;
    std::vector<int32_t> hdr, buf;
    for (size_t c0 = 0; c0 < cand.size(); c0 += chunk) {
        const int32_t cnt = (int32_t)std::min<size_t>(chunk, cand.size() - c0);
        if (!hip_ok(hipMemcpyAsync(cslots, cand.data() + c0, (size_t)cnt * 4, hipMemcpyHostToDevice, s), "paths copy"))
            return APSP_E_DEVICE;
        g->prof.begin(KID_QUERY);
        SR(g, launch_query_paths)(g->dg, si, sj, cslots, cnt, qout, qsc, s);
        g->prof.end();
        if ((st = check_launch("apsp_query_paths"))) return st;
        // the 2 cnt headers (dist, length, status), then the paths up to the longest
        const size_t pitch = (size_t)(P + 3) * 4;
        hdr.resize((size_t)2 * cnt * 3);
        if (!hip_ok(hipMemcpy2DAsync(hdr.data(), 12, qout, pitch, 12, 2 * cnt, hipMemcpyDeviceToHost, s), "paths read") ||
            !hip_ok(hipStreamSynchronize(s), "paths sync"))
            return APSP_E_DEVICE;
        int32_t longest = 0;
        for (int32_t q = 0; q < 2 * cnt; ++q) {
            if (hdr[3 * q + 2] != 0) return fail(APSP_E_DEVICE, "apsp_query_paths: no shortest path found on the device");
            longest = std::max(longest, hdr[3 * q + 1]);
        }
        const size_t w = (size_t)(3 + longest) * 4;
        buf.resize((size_t)2 * cnt * (3 + longest));
        if (!hip_ok(hipMemcpy2DAsync(buf.data(), w, qout, pitch, w, 2 * cnt, hipMemcpyDeviceToHost, s), "paths read") ||
            !hip_ok(hipStreamSynchronize(s), "paths sync"))
            return APSP_E_DEVICE;
        for (int32_t c = 0; c < cnt; ++c) {
            const int32_t *a = buf.data() + (size_t)(2 * c) * (3 + longest);
            const int32_t *b = buf.data() + (size_t)(2 * c + 1) * (3 + longest);
            std::vector<int32_t> p(a + 3, a + 3 + a[1]);   // i -> t
            p.insert(p.end(), b + 4, b + 3 + b[1]);         // t -> j without t
            if (seen.insert(p).second) paths.push_back(std::move(p));
        }
    }
    int64_t total = 0;
    for (const auto &p : paths) total += (int64_t)p.size();
    *npaths = (int32_t)paths.size();
    *ids_len = total;
    if (offsets_cap < (int32_t)paths.size() + 1 || ids_cap < total)
        return fail(APSP_E_CAPACITY, "apsp_query_paths: output too small (npaths and ids_len give the sizes)");
    int64_t off = 0;
    for (size_t q = 0; q < paths.size(); ++q) {
        offsets[q] = (int32_t)off;
        std::copy(paths[q].begin(), paths[q].end(), ids + off);
        off += (int64_t)paths[q].size();
    }
    offsets[paths.size()] = (int32_t)off;
    return APSP_OK;
}

apsp_status apsp_read_matrix(apsp_graph *g, int32_t *out_dev, int64_t out_ld) {
    if (!g) return fail(APSP_E_INVALID, "apsp_read_matrix: NULL graph");
    if (g->detached) return detached_error("apsp_read_matrix");
    if (g->n_live > 0 && (!out_dev || out_ld < g->n_live)) return fail(APSP_E_INVALID, "apsp_read_matrix: bad output");
    launch_gather_compact(g->dg.D, g->dg.ld, out_dev, out_ld, g->rank_cur, g->n_live, g->dg.widest, g->stream);
    return check_launch("apsp_read_matrix");
}

apsp_status apsp_read_adjacency(apsp_graph *g, int32_t *out_dev, int64_t out_ld) {
    if (!g) return fail(APSP_E_INVALID, "apsp_read_adjacency: NULL graph");
    if (g->detached) return detached_error("apsp_read_adjacency");
    if (g->n_live > 0 && (!out_dev || out_ld < g->n_live))
        return fail(APSP_E_INVALID, "apsp_read_adjacency: bad output");
    launch_gather_compact(g->dg.A, g->dg.ld, out_dev, out_ld, g->rank_cur, g->n_live, g->dg.widest, g->stream);
    return check_launch("apsp_read_adjacency");
}

apsp_status apsp_next_id(const apsp_graph *g, int32_t *id) {
    if (!g || !id) return fail(APSP_E_INVALID, "apsp_next_id: NULL argument");
    *id = g->max_id + 1;
    return APSP_OK;
}

apsp_status apsp_node_count(const apsp_graph *g, int32_t *n) {
    if (!g || !n) return fail(APSP_E_INVALID, "apsp_node_count: NULL argument");
    *n = g->n_live;
    return APSP_OK;
}

apsp_status apsp_node_ids(const apsp_graph *g, int32_t *ids, int32_t cap, int32_t *n) {
    if (!g || !n || cap < 0 || (cap > 0 && !ids)) return fail(APSP_E_INVALID, "apsp_node_ids: bad argument");
    *n = g->n_live;
    if (cap < g->n_live) return fail(APSP_E_CAPACITY, "apsp_node_ids: cap too small");
    std::copy(g->live_ids.begin(), g->live_ids.end(), ids);
    return APSP_OK;
}

apsp_status apsp_edge_scope(apsp_graph *g, int32_t u, int32_t v, int32_t *r_count, int32_t *c_count) {
    if (!g || !r_count || !c_count) return fail(APSP_E_INVALID, "apsp_edge_scope: NULL argument");
    if (g->detached) return detached_error("apsp_edge_scope");
    if (u == v) return fail(APSP_E_INVALID, "apsp_edge_scope: u == v");
    int32_t su, sv;
    if (!lookup(g, u, &su) || !lookup(g, v, &sv)) return fail(APSP_E_NOT_FOUND, "apsp_edge_scope: id is not live");
    launch_fill(&g->dg.ctl->scope_r, 2, 0, g->stream);
    SR(g, launch_edge_scope)(g->dg, su, sv, g->stream);
    apsp_status st = check_launch("apsp_edge_scope");
    if (st) return st;
    if ((st = read_ctl(g))) return st;
    *r_count = g->ctl_h->scope_r;
    *c_count = g->ctl_h->scope_c;
    return APSP_OK;
}

apsp_status apsp_last_stats(apsp_graph *g, apsp_update_stats *out) {
    if (!g || !out) return fail(APSP_E_INVALID, "apsp_last_stats: NULL argument");
    if (g->detached) return detached_error("apsp_last_stats");
    apsp_status st = flush_stats(g);
    if (!st) st = read_ctl(g);
    if (st) return st;
    const Ctl &c = *g->ctl_h;
    std::memset(out, 0, sizeof(*out));
    out->flagged = (int64_t)c.flagged;
    out->rows = c.rows;
    out->n_before = g->last_n_before;
    out->full_scans = c.full_scans;
    out->sweeps = c.sweeps;
    out->rows_relaxed = c.rows_relaxed;
    out->heavy_rows = c.heavy_count;
    out->rows_changed = c.rows_changed;
    out->changed = (int64_t)c.changed;
    out->fallback = g->last_fallback;
    int32_t kind = g->last_kind;
    if (kind == -1) {  // edge update: the device chose the path
        kind = c.edge_mode == EDGE_INCREASE ? UK_INCREASE : (c.edge_mode == EDGE_DECREASE ? UK_DECREASE : UK_NONE);
        out->noop = c.edge_mode == EDGE_NOOP;
    }
    out->kind = kind;
    if (kind == UK_REMOVE || kind == UK_INCREASE) {
        out->cost = g->last_n_before > 1 ? (double)c.rows / (double)(g->last_n_before - 1) : 0.0;
        out->cost_refined = g->last_n_before > 1 ? (double)c.rows_changed / (double)(g->last_n_before - 1) : 0.0;
    }
    if (kind == UK_REMOVE) out->noop = c.flagged == 0 && !g->last_fallback;
    out->route = (kind == UK_REMOVE || kind == UK_INCREASE) ? g->last_route : 0;
    return APSP_OK;
}

apsp_status apsp_sync(apsp_graph *g) {
    if (!g) return fail(APSP_E_INVALID, "apsp_sync: NULL graph");
    if (g->detached) return detached_error("apsp_sync");
    apsp_status st = read_ctl(g);
    if (st) return st;
    if (g->ctl_h->err) {
        launch_fill(&g->dg.ctl->err, 1, 0, g->stream);
        if (!hip_ok(hipStreamSynchronize(g->stream), "stream sync")) return APSP_E_DEVICE;
        return fail(APSP_E_VALUE, "a device-resident weight was outside [0, APSP_INF]; it was treated as an absent edge");
    }
    return APSP_OK;
}

apsp_status apsp_profile_every(apsp_graph *g, int64_t kernel_mask, int32_t every) {
    if (!g) return fail(APSP_E_INVALID, "apsp_profile: NULL graph");
    if (every < 1) return fail(APSP_E_INVALID, "apsp_profile_every: every must be at least 1");
    if (!hip_ok(hipStreamSynchronize(g->stream), "stream sync")) return APSP_E_DEVICE;
    g->prof_impl.collect();
    for (int k = 0; k < KID_COUNT; ++k) {
        g->prof_impl.count[k] = 0;
        g->prof_impl.ms[k] = 0.0;
        g->prof_impl.seen[k] = 0;
    }
    g->prof_impl.mask = kernel_mask;
    g->prof_impl.every = every;
    g->prof.on = kernel_mask != 0;
    return APSP_OK;
}

apsp_status apsp_profile(apsp_graph *g, int64_t kernel_mask) { return apsp_profile_every(g, kernel_mask, 1); }

apsp_status apsp_profile_read(apsp_graph *g, int32_t kernel, int64_t *launches, double *total_ms) {
    if (!g || !launches || !total_ms) return fail(APSP_E_INVALID, "apsp_profile_read: NULL argument");
    if (kernel < 0 || kernel >= KID_COUNT) return fail(APSP_E_INVALID, "apsp_profile_read: bad kernel id");
    if (!hip_ok(hipStreamSynchronize(g->stream), "stream sync")) return APSP_E_DEVICE;
    g->prof_impl.collect();
    *launches = g->prof_impl.count[kernel];
    *total_ms = g->prof_impl.ms[kernel];
    return APSP_OK;
}

}  // extern "C"
