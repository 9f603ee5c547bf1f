// Host-side state of a graph handle and the helpers the C ABI's units share:
// the device buffer layout, the id <-> slot map, and error reporting.
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>
#include <set>
#include <string>
#include <unordered_map>
#include <vector>

#include "apsp_internal.h"

namespace apsp_host {

using namespace apsp;

extern thread_local std::string g_err;

inline apsp_status fail(apsp_status st, const std::string &msg) {
    g_err = msg;
    return st;
}

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

inline int32_t padded(int32_t cap) { return ((cap + TILE - 1) / TILE) * TILE; }

struct Layout {
    size_t D, A, AT, nin, nin_cnt, nin_beta, id_of_slot, vec, plist, rank_a, rank_b, qbuf, qscratch, fscratch,
        nin_queue, heavy_rows, heavy_epoch, flag_bits, row_bits, marks, partials, ctl, total;
};

constexpr int NVEC = 8;  // wo, wi, out, in, colu, colv, rowu, rowv

inline Layout make_layout(int32_t cap, int32_t kind) {
    Layout L{};
    const size_t P = (size_t)padded(cap);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off = align256(off + bytes);
        return o;
    };
    const size_t mat = P * P * sizeof(int32_t);
    L.D = take(mat);
    L.A = take(mat);
    L.AT = kind == APSP_DIRECTED ? take(mat) : (size_t)-1;
    L.nin = take(P * NIN_L * sizeof(int2));
    L.nin_cnt = take(P * 4);
    L.nin_beta = take(P * 4);
    L.id_of_slot = take(P * 4);
    L.vec = take((size_t)NVEC * P * 4);
    L.plist = take(NIN_L * sizeof(int2) + 256);
    L.rank_a = take(P * 4);
    L.rank_b = take(P * 4);
    L.qbuf = take((P + 8) * 4);
    L.qscratch = take(4 * P * 4);
    L.fscratch = take((size_t)FUSED_GRID * 2 * P * 4);
    L.nin_queue = take(P * 4);
    L.heavy_rows = take(P * 4);
    L.heavy_epoch = take(P * 4);
    L.flag_bits = take(P * ((P + 31) / 32) * 4);
    L.row_bits = take(((P + 31) / 32) * 4);
    L.marks = take((P / 8) * mark_pitch(P));
    L.partials = take(((size_t)RECOMPUTE_BLOCKS * RECOMPUTE_STATS + 2 * (size_t)FUSED_GRID) * 4);
    L.ctl = take(sizeof(Ctl));
    L.total = off;
    return L;
}

enum UpdateKind { UK_NONE = 0, UK_ADD = 1, UK_REMOVE = 2, UK_DECREASE = 3, UK_INCREASE = 4 };

struct ProfImpl {
    hipStream_t stream = nullptr;
    int64_t mask = 0;
    std::vector<hipEvent_t> pool;
    size_t used = 0;
    struct Rec {
        int32_t kid;
        hipEvent_t a, b;
    };
    std::vector<Rec> recs;
    int32_t cur_kid = -1;
    hipEvent_t cur_a = nullptr;
    int64_t count[KID_COUNT] = {};
    double ms[KID_COUNT] = {};
    int64_t seen[KID_COUNT] = {};  // launches of each kernel since apsp_profile_every
    int32_t every = 1;

    hipEvent_t take() {
        if (used == pool.size()) {
            hipEvent_t e;
            if (hipEventCreate(&e) != hipSuccess) return nullptr;
            pool.push_back(e);
        }
        return pool[used++];
    }
    void collect() {
        for (auto &r : recs) {
            float t = 0.f;
            if (hipEventElapsedTime(&t, r.a, r.b) == hipSuccess) {
                count[r.kid] += 1;
                ms[r.kid] += t;
            }
        }
        recs.clear();
        used = 0;
    }
    ~ProfImpl() {
        for (auto e : pool) (void)hipEventDestroy(e);
    }
};

}  // namespace apsp_host

struct apsp_graph {
    using ProfImpl = apsp_host::ProfImpl;
    int32_t cap = 0, P = 0, kind = 0;  // kind: APSP_DIRECTED or APSP_UNDIRECTED
    int32_t minimax = 0;                // the (min, max) semiring (APSP_MINIMAX)
    hipStream_t stream = nullptr;
    char *base = nullptr;
    apsp::DevGraph dg{};
    int32_t *vec[apsp_host::NVEC] = {};
    int2 *plist = nullptr;
    int32_t *plist_cnt = nullptr, *plist_beta = nullptr;
    int32_t *rank_cur = nullptr, *rank_other = nullptr;
    int32_t *qbuf = nullptr, *qscratch = nullptr, *fscratch = nullptr, *nin_queue = nullptr;
    int32_t *heavy_rows = nullptr, *heavy_epoch = nullptr;
    uint32_t *flag_bits = nullptr, *row_bits = nullptr;
    uint8_t *marks = nullptr;
    int32_t *partials = nullptr;
    int32_t epoch = 0;
    // set by apsp_graph_detach (the device buffer is no longer the graph's),
    // cleared by apsp_graph_relocate; every call that would touch device
    // memory refuses a detached graph
    int32_t detached = 0;
    // host bookkeeping
    int32_t n_live = 0, max_id = -1;
    std::vector<int32_t> live_ids;  // ascending
    std::unordered_map<int32_t, int32_t> slot_of_id;
    std::set<int32_t> free_slots;
    int32_t policy = APSP_FALLBACK_NEVER;
    double delta = 0.5;
    int32_t last_kind = apsp_host::UK_NONE, last_n_before = 0, last_fallback = 0;
    int32_t last_route = 0;  // 1: the last removal or tight increase took the spanning-forest route
    // nonzero: the last update was an edge update whose recompute statistics
    // are still per-work-group partials (this many work-groups, as
    // launch_mask_recompute returned); summed into ctl before ctl is read
    int32_t stats_pending = 0;
    apsp::Ctl *ctl_h = nullptr;   // pinned
    int32_t *qbuf_h = nullptr;  // pinned
    ProfImpl prof_impl;
    apsp::Prof prof;
};

namespace apsp_host {

inline bool hip_ok(hipError_t e, const char *what) {
    if (e == hipSuccess) return true;
    g_err = std::string(what) + ": " + hipGetErrorString(e);
    return false;
}

inline apsp_status check_launch(const char *what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(APSP_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
    return APSP_OK;
}

inline int32_t *&wo(apsp_graph *g) { return g->vec[0]; }
inline int32_t *&wi(apsp_graph *g) { return g->vec[1]; }
inline int32_t *&vout(apsp_graph *g) { return g->vec[2]; }
inline int32_t *&vin(apsp_graph *g) { return g->vec[3]; }
inline int32_t *&colu(apsp_graph *g) { return g->vec[4]; }
inline int32_t *&colv(apsp_graph *g) { return g->vec[5]; }
inline int32_t *&rowu(apsp_graph *g) { return g->vec[6]; }
inline int32_t *&rowv(apsp_graph *g) { return g->vec[7]; }

inline int32_t rank_of(const apsp_graph *g, int32_t id) {
    auto it = std::lower_bound(g->live_ids.begin(), g->live_ids.end(), id);
    if (it == g->live_ids.end() || *it != id) return -1;
    return (int32_t)(it - g->live_ids.begin());
}

// The error every device-touching call returns for a detached graph.
inline apsp_status detached_error(const char *who) {
    return fail(APSP_E_INVALID, std::string(who) +
                                    ": the graph is detached from device memory (apsp_graph_detach); "
                                    "apsp_graph_relocate gives it a buffer again");
}

inline bool lookup(const apsp_graph *g, int32_t id, int32_t *slot) {
    auto it = g->slot_of_id.find(id);
    if (it == g->slot_of_id.end()) return false;
    *slot = it->second;
    return true;
}

// The working memory of one edge update (device pointers): gathered columns
// and rows of u and v, the heavy-row pass scratch (FUSED_GRID * 2 * P ints),
// its row list and epoch marks (P ints each; heavy_epoch[i] == epoch marks a
// heavy row, so epochs must not repeat on one array), the flag bitmap
// (P * ceil(P/32) words, zero on entry), row bits (ceil(P/32) words, zero on
// entry), row marks ((P/8) * mark_pitch(P) bytes) and the recompute's
// per-work-group statistics.
struct EdgeScratch {
    int32_t *colu, *colv, *rowu, *rowv;
    int32_t *fscratch, *heavy_rows, *heavy_epoch;
    uint32_t *flag_bits, *row_bits;
    uint8_t *marks;
    int32_t *partials;
    int32_t epoch;
    // partials in the graph's own memory: summed when the statistics are read
    bool lazy_stats = false;
};

// Argument checks of an edge update (nothing enqueued); slots of u and v.
apsp_status check_edge_args(apsp_graph *g, const char *who, int32_t u, int32_t v, int32_t w, int32_t *su,
                            int32_t *sv);
// An edge update over the given working memory (apsp_update_edge passes the
// graph's own; the no-allocation variant passes the library's static array).
apsp_status update_edge_with(apsp_graph *g, const char *who, int32_t u, int32_t v, int32_t w,
                             const EdgeScratch &sc);

}  // namespace apsp_host
