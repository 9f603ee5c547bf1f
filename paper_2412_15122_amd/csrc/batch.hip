// Batched updates over many graphs.
//
// Each update runs the same method as the single-graph kernels:
//   add node     Corollaries 1 / 2 (new row / column over
//                the new node's light edges) and Theorem 3 (relaxation)
//   remove node  Corollary 3 mask, then Bellman-Ford recompute of
//                the flagged entries of each row (one wavefront per row)
//   edge update  decrease: relaxation through the new edge; increase: mask
//                of the pairs that can use the edge, then the same recompute
//   query        Algorithm 7 (candidates, then the canonical walk)
// split into phases: a prologue and an epilogue that one work-group runs per
// graph (list selection, O(n) vectors, placement, index edits), and row
// sweeps (relaxation, mask, recompute) that any number of work-groups can
// share by row ranges.
//
// Two schedules over the same phases:
//   work queue  every work-group pops a graph (most work first) and runs all
//               of its items, every phase, alone; no waiting between
//               work-groups.  Good for many small graphs.
//   lockstep    step s applies item s of every graph: graph-parallel
//               epilogue(s-1) + prologue(s), then the row sweeps of all
//               graphs spread over the whole grid, with grid barriers between
//               the phases.  The grid is launched cooperatively (all of it
//               resident); every barrier wait is bounded and a timeout is
//               reported instead of hanging.  Good when large graphs would
//               leave one work-group streaming a whole matrix.
#include <algorithm>

#include "batch_internal.h"
#include "device_common.h"

namespace apsp {
APSP_SR_BEGIN

// ---------------------------------------------------------------------------
// streaming helpers
// ---------------------------------------------------------------------------

// Two 4-column slices of the row vectors a sweep tests against.
struct Vec2 {
    uint4 a, b;
};

// Visits the 4-column groups of rows [r0, r1) (columns [0, n)) whose
// row_ok(i) holds.  A wavefront takes one 256-column chunk (64 lanes x 4
// columns) of U consecutive rows at a time: it reads the chunk's slice of the
// row vectors once (vecs(c0)), then issues the U rows' 16-byte loads of D
// (non-temporal: streamed once) together before it uses any.  body(i, c0,
// ok, d, v) runs on every lane (ok false where the lane has no group), so it
// may use cross-lane operations; after the U rows, piece_end(i0) runs on
// every lane of the wavefront.
struct NoPieceEnd {
    __device__ void operator()(int32_t) const {}
};

template <int U, class RowOk, class Vecs, class Body, class PieceEnd = NoPieceEnd>
__device__ inline void stream_chunks(const DevGraph &g, int32_t n, int32_t r0, int32_t r1, RowOk row_ok, Vecs vecs,
                                     Body body, PieceEnd piece_end = PieceEnd()) {
    const int lane = lane_id(), wv = threadIdx.x >> 6;
    const int32_t Q = (n + 255) >> 8;
    const int32_t total = ((r1 - r0 + U - 1) / U) * Q;
    for (int32_t k = wv; k < total; k += BATCH_THREADS / 64) {
        const int32_t i0 = r0 + (k / Q) * U;
        const int32_t c0 = (k % Q) * 256 + lane * 4;
        const bool col_ok = c0 < n;
        bool ok[U];
        bool any = false;
#pragma unroll
        for (int u = 0; u < U; ++u) {
            ok[u] = i0 + u < r1 && row_ok(i0 + u);
            any = any || ok[u];
        }
        if (!any) continue;  // wave-uniform
        const Vec2 v = vecs(c0);
        uint4 d[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            ok[u] = ok[u] && col_ok;
            d[u] = make_uint4(INF, INF, INF, INF);
            if (ok[u]) d[u] = load_stream4(g.D + (int64_t)(i0 + u) * g.ld + c0);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) body(i0 + u, c0, ok[u], d[u], v);
        piece_end(i0);
    }
}

// stage[0..n) = a[0..n) and stage[P..P+n) = b[0..n) (b may be null), padded
// with INF to a multiple of 4.
__device__ inline void stage_rows(uint32_t *stage, int32_t P, int32_t n, const int32_t *a, const int32_t *b) {
    const int32_t n4 = (n + 3) & ~3;
    for (int32_t c = threadIdx.x; c < n4; c += BATCH_THREADS) {
        stage[c] = c < n ? (uint32_t)a[c] : INF;
        if (b) stage[P + c] = c < n ? (uint32_t)b[c] : INF;
    }
    __syncthreads();
}

// 4 consecutive entries of a row vector (16-byte aligned at c0; columns >= n
// read as INF; one 16-byte load away from the tail).
__device__ inline uint4 vec4(const uint32_t *v, int32_t c0, int32_t n) {
    if (c0 + 3 < n) return *reinterpret_cast<const uint4 *>(v + c0);
    return make_uint4(c0 < n ? v[c0] : INF, c0 + 1 < n ? v[c0 + 1] : INF, c0 + 2 < n ? v[c0 + 2] : INF,
                      c0 + 3 < n ? v[c0 + 3] : INF);
}

// D[i][c0..c0+3] := min(D, t), stored only when something changed.
__device__ inline void store_min4(const DevGraph &g, int32_t i, int32_t c0, uint4 d, uint4 t) {
    if (t.x < d.x || t.y < d.y || t.z < d.z || t.w < d.w) {
        d.x = min(d.x, t.x);
        d.y = min(d.y, t.y);
        d.z = min(d.z, t.z);
        d.w = min(d.w, t.w);
        *reinterpret_cast<uint4 *>(g.D + (int64_t)i * g.ld + c0) = d;
    }
}

// ---------------------------------------------------------------------------
// add node
// ---------------------------------------------------------------------------

// Weights by slot and the new node's light lists: its in-edges in the index
// (from wi) and, for a directed graph, its out-edges in plist (from wo).
__device__ __forceinline__ void add_setup(const DevGraph &g, const BatchGraph &bg, const BatchItem &it, SelectShared &ssh,
                                          uint32_t *stage) {
    const int tid = threadIdx.x;
    const int n = g.n_slots;
    const int32_t p = it.a, rank = it.c;
    const bool und = g.undirected != 0;
    int32_t *wo = bg.wo;
    int32_t *wi = und ? bg.wo : bg.wi;
    for (int32_t s = tid; s < n; s += BATCH_THREADS) {
        wo[s] = (int32_t)INF;
        wi[s] = (int32_t)INF;
    }
    __syncthreads();
    for (int32_t r = tid; r < rank; r += BATCH_THREADS) {
        const int32_t s = it.rank_src[r];
        int32_t a = it.w_out[r];
        int32_t b = und ? a : it.w_in[r];
        int bad = 0;
        if (a < 0 || (uint32_t)a > INF) { a = (int32_t)INF; bad = 1; }
        if (b < 0 || (uint32_t)b > INF) { b = (int32_t)INF; bad = 1; }
        if (g.widest) {
            a = widest_xf(a);
            b = widest_xf(b);
        }
        wo[s] = a;
        wi[s] = b;
        if (bad) atomicOr(&g.ctl->err, (int32_t)ERR_VALUE);
    }
    __syncthreads();
    int2 *pin = g.nin + (int64_t)p * NIN_L;
    select_light(wi, n, p, pin, g.nin_cnt + p, g.nin_beta + p, ssh, stage);
    if (!und) select_light(wo, n, p, bg.plist, bg.plist_cnt, bg.plist_beta, ssh, stage);
    __syncthreads();
}

// The new row over the 256 columns [cb, cb + 256): out[c] = min_t wo[t] +
// D[t][c] (Corollary 1).  The 4 waves split p's out-list (ascending
// weight; a wave stops once the next weight reaches every value it holds,
// distances being >= 0); every unlisted t has wo[t] >= the list bound, so a
// column at or below it is final, and the others take an exhaustive scan.
__device__ __forceinline__ void add_out_cols(const DevGraph &g, const BatchGraph &bg, const BatchItem &it, int32_t cb) {
    __shared__ uint32_t s_part[4][256];
    __shared__ uint32_t s_red[32];
    const int n = g.n_slots;
    const int tid = threadIdx.x, lane = lane_id(), wv = tid >> 6;
    const int32_t p = it.a;
    const bool und = g.undirected != 0;
    const int2 *ol = und ? g.nin + (int64_t)p * NIN_L : bg.plist;
    const int ocnt = und ? g.nin_cnt[p] : *bg.plist_cnt;
    const uint32_t obeta = (uint32_t)(und ? g.nin_beta[p] : *bg.plist_beta);
    const int lim = min(ocnt, g.lim);
    const uint32_t beta_eff = ocnt > g.lim ? (uint32_t)ol[g.lim].y : obeta;
    const int32_t c0 = cb + lane * 4;
    bool live[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) live[e] = c0 + e < n && g.id_of_slot[c0 + e] >= 0;
    uint32_t acc[4] = {INF, INF, INF, INF};
    if (c0 < n) {
        // the wavefront's entries wv, wv + 4, ... four at a time: their rows'
        // loads are in flight together; it stops at the first entry that
        // weighs at least every value it holds
        for (int e0 = wv; e0 < lim; e0 += 16) {
            uint32_t mx = 0;
#pragma unroll
            for (int q = 0; q < 4; ++q)
                if (live[q]) mx = max(mx, acc[q]);
            int2 ent[4];
            uint4 v[4];
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int e = e0 + 4 * t;
                ent[t] = e < lim ? ol[e] : make_int2(0, (int)INF);
                v[t] = make_uint4(INF, INF, INF, INF);
                if ((uint32_t)ent[t].y < mx)
                    v[t] = vec4(reinterpret_cast<const uint32_t *>(g.D + (int64_t)ent[t].x * g.ld), c0, n);
            }
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const uint32_t w = (uint32_t)ent[t].y;
                acc[0] = min(acc[0], cat(w, v[t].x));
                acc[1] = min(acc[1], cat(w, v[t].y));
                acc[2] = min(acc[2], cat(w, v[t].z));
                acc[3] = min(acc[3], cat(w, v[t].w));
            }
            if ((uint32_t)ent[3].y >= mx) break;  // every later entry is at least as heavy
        }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) s_part[wv][lane * 4 + q] = acc[q];
    __syncthreads();
    const int32_t c = cb + tid;  // one column per thread from here on
    uint32_t fin = min(min(s_part[0][tid], s_part[1][tid]), min(s_part[2][tid], s_part[3][tid]));
    const bool live_c = c < n && g.id_of_slot[c] >= 0;
    const int need = block_sum<BATCH_THREADS>(live_c && fin > beta_eff, s_red);
    if (need && live_c && fin > beta_eff)
        for (int32_t t = 0; t < n; ++t) fin = min(fin, cat((uint32_t)bg.wo[t], (uint32_t)g.D[(int64_t)t * g.ld + c]));
    if (c < n) bg.vout[c] = live_c ? (int32_t)min(fin, INF) : (int32_t)INF;
    __syncthreads();
}

// The new column over rows [r0, r1) (directed graphs): in[r] = min_x D[r][x] (+)
// wi[x] (Corollary 2), over p's light in-edges (at most 64, read
// once per wavefront: lane l of a 16-lane group holds entries l, l + 16,
// l + 32, l + 48).  A wavefront takes 4 rows at a time, one per 16-lane
// group, each lane's 4 gathers of the row in flight together; a row whose
// value exceeds the list bound then gets an exhaustive scan by the whole
// wavefront.  Values go to bg.vin and, when rows_out is set, to
// rows_out[r - r0] as well.
__device__ __forceinline__ void add_in_rows(const DevGraph &g, const BatchGraph &bg, const BatchItem &it, int32_t r0,
                                            int32_t r1, uint32_t *rows_out = nullptr) {
    const int lane = lane_id(), wv = threadIdx.x >> 6;
    const int sub = lane >> 4, l16 = lane & 15;
    const int32_t p = it.a;
    const int2 *L = g.nin + (int64_t)p * NIN_L;
    const int cnt = g.nin_cnt[p];
    const int lim = min(cnt, g.lim);
    const uint32_t beta_eff = cnt > g.lim ? (uint32_t)L[g.lim].y : (uint32_t)g.nin_beta[p];
    int2 ent[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int e = l16 + 16 * q;
        ent[q] = e < lim ? L[e] : make_int2(0, (int)INF);
    }
    for (int32_t rb = r0 + wv * 4; rb < r1; rb += BATCH_THREADS / 16) {
        const int32_t r = rb + sub;
        const bool live = r < r1 && g.id_of_slot[r] >= 0;
        uint32_t best = INF;
        if (live) {
            const int32_t *Dr = g.D + (int64_t)r * g.ld;
            uint32_t v[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) v[q] = (uint32_t)ent[q].y < INF ? (uint32_t)Dr[ent[q].x] : INF;
#pragma unroll
            for (int q = 0; q < 4; ++q)
                if ((uint32_t)ent[q].y < INF) best = min(best, cat((uint32_t)ent[q].y, v[q]));
        }
#pragma unroll
        for (int o = 1; o < 16; o <<= 1) best = min(best, (uint32_t)__shfl_xor((int)best, o, 16));
        unsigned long long m = __ballot(live && l16 == 0 && best > beta_eff);
        while (m) {  // wave-uniform
            const int b = __ffsll((long long)m) - 1;
            m &= m - 1;
            // only in-weights below the row's current value can lower it
            const uint32_t cur = (uint32_t)__shfl((int)best, b);
            const uint32_t x_best = wave_min_plus_below(g.D + (int64_t)(rb + (b >> 4)) * g.ld, bg.wi, g.n_slots, cur);
            if (lane == b) best = min(best, x_best);
        }
        if (r < r1 && l16 == 0) {
            const int32_t val = live ? (int32_t)min(best, INF) : (int32_t)INF;
            bg.vin[r] = val;
            if (rows_out) rows_out[r - r0] = (uint32_t)val;
        }
    }
}

// Chunk c of an add's vector phase (add_vec_chunks).
__device__ __forceinline__ void add_vec_chunk(const DevGraph &g, const BatchGraph &bg, const BatchItem &it, int32_t c) {
    const int32_t no = add_out_chunks(g.n_slots);
    if (c < no) {
        add_out_cols(g, bg, it, c * 256);
    } else {
        const int32_t r0 = (c - no) * ADD_IN_ROWS;
        add_in_rows(g, bg, it, r0, min(r0 + ADD_IN_ROWS, g.n_slots));
    }
}

// The whole add prologue by one work-group (work-queue schedule).
__device__ __forceinline__ void add_prologue(const DevGraph &g, const BatchGraph &bg, const BatchItem &it, SelectShared &ssh,
                                             uint32_t *stage) {
    add_setup(g, bg, it, ssh, stage);
    const int32_t nc = add_vec_chunks(g.n_slots, g.undirected != 0);
    for (int32_t c = 0; c < nc; ++c) add_vec_chunk(g, bg, it, c);
    __syncthreads();
}

// Theorem 3 over rows [r0, r1): D[i][j] = min(D[i][j], in[i] (+) out[j]).
// outv: the new row (LDS stage or global); in_of(i): in[i] (from the graph's
// vector or an LDS copy of the chunk's rows).
template <int U, class InOf>
__device__ __forceinline__ void add_relax_rows(const DevGraph &g, const BatchGraph &bg, int32_t r0, int32_t r1, const uint32_t *outv,
                                               InOf in_of) {
    const int n = g.n_slots;
    stream_chunks<U>(
        g, n, r0, r1, [&](int32_t i) { return in_of(i) < INF; },
        [&](int32_t c0) { return Vec2{vec4(outv, c0, n), make_uint4(0, 0, 0, 0)}; },
        [&](int32_t i, int32_t c0, bool ok, uint4 d, const Vec2 &v) {
            if (!ok) return;
            const uint32_t a = in_of(i);
            const uint4 o = v.a;
            store_min4(g, i, c0, d, make_uint4(cat(a, o.x), cat(a, o.y), cat(a, o.z), cat(a, o.w)));
        });
}

// Index-list edits four lists at a time (an epilogue edits up to a few
// percent of all lists, each a round trip when done one by one): the
// lists' entries, counts and bounds are read together, then each list is
// edited from the registers with the single-list logic of
// wave_list_insert / wave_list_purge.  The lists must differ.
struct ListRegs {
    int2 ent;  // entry `lane` (every list has NIN_L slots)
    int cnt;
    uint32_t beta;
};

__device__ __forceinline__ ListRegs list_load(const DevGraph &g, int32_t y) {
    ListRegs r;
    r.ent = g.nin[(int64_t)y * NIN_L + lane_id()];
    r.cnt = g.nin_cnt[y];
    r.beta = (uint32_t)g.nin_beta[y];
    return r;
}

__device__ __forceinline__ void list_insert_regs(const DevGraph &g, int32_t y, const ListRegs &r, int32_t x,
                                                 uint32_t w) {
    const int lane = lane_id();
    if (w >= INF || w >= r.beta) return;
    const int cnt = r.cnt;
    const int2 ent = lane < cnt ? r.ent : make_int2(0, (int)INF);
    const int pos = __popcll(__ballot(lane < cnt && (uint32_t)ent.y <= w));
    const int px = __shfl_up(ent.x, 1), py = __shfl_up(ent.y, 1);
    const int ncnt = min(cnt + 1, NIN_L);
    uint32_t dropped = INF;
    if (cnt == NIN_L) dropped = (pos < NIN_L) ? (uint32_t)__shfl(ent.y, NIN_L - 1) : w;
    const int2 ne = lane < pos ? ent : (lane == pos ? make_int2(x, (int)w) : make_int2(px, py));
    if (lane < ncnt) g.nin[(int64_t)y * NIN_L + lane] = ne;
    if (lane == 0) {
        g.nin_cnt[y] = ncnt;
        if (cnt == NIN_L) g.nin_beta[y] = (int32_t)min(r.beta, dropped);
    }
}

__device__ __forceinline__ void list_purge_regs(const DevGraph &g, int32_t y, const ListRegs &r, int32_t x) {
    const int lane = lane_id();
    const int cnt = r.cnt;
    const int2 ent = lane < cnt ? r.ent : make_int2(0, (int)INF);
    const unsigned long long m = __ballot(lane < cnt && ent.x == x);
    if (m == 0) return;
    const int pos = __ffsll((long long)m) - 1;
    const int nx = __shfl_down(ent.x, 1), ny = __shfl_down(ent.y, 1);
    int2 *L = g.nin + (int64_t)y * NIN_L;
    if (lane >= pos && lane < cnt - 1) L[lane] = make_int2(nx, ny);
    if (lane == cnt - 1) L[lane] = make_int2(0, (int)INF);
    if (lane == 0) g.nin_cnt[y] = cnt - 1;
}

// The next (up to) four set bits of the wave-uniform mask m as lists
// y0 + bit (-1 where none is left).
__device__ __forceinline__ void take4(unsigned long long &m, int32_t y0, int32_t (&yq)[4]) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        yq[q] = -1;
        if (m) {
            yq[q] = y0 + __ffsll((long long)m) - 1;
            m &= m - 1;
        }
    }
}

// Row and column p of D, A (and A^T), the id, the rank, and p's out-edges in
// every other node's light list.
__device__ __forceinline__ void add_epilogue(const DevGraph &g, const BatchGraph &bg, const BatchItem &it) {
    const int tid = threadIdx.x;
    const int n = g.n_slots;
    const int32_t p = it.a, new_id = it.b, rank = it.c;
    const bool und = g.undirected != 0;
    const int32_t *wo = bg.wo;
    const int32_t *wi = und ? bg.wo : bg.wi;
    const int32_t *in = und ? bg.vout : bg.vin;
    const int32_t *out = bg.vout;
    const int64_t ld = g.ld;
    for (int32_t s = tid; s < n; s += BATCH_THREADS) {
        if (s == p) continue;
        g.D[(int64_t)p * ld + s] = out[s];
        g.D[(int64_t)s * ld + p] = in[s];
        g.A[(int64_t)p * ld + s] = wo[s];
        g.A[(int64_t)s * ld + p] = wi[s];
        if (!und) {
            g.AT[(int64_t)s * ld + p] = wo[s];
            g.AT[(int64_t)p * ld + s] = wi[s];
        }
    }
    if (tid == 0) {
        g.D[(int64_t)p * ld + p] = 0;
        g.A[(int64_t)p * ld + p] = 0;
        if (!und) g.AT[(int64_t)p * ld + p] = 0;
        g.id_of_slot[p] = new_id;
        it.rank_src[rank] = p;
    }
    __syncthreads();
    // lanes screen 64 lists at a time: an edge at or above a list's bound is
    // not listed
    for (int32_t y0 = (tid >> 6) * 64; y0 < n; y0 += BATCH_THREADS) {
        const int32_t y = y0 + lane_id();
        const bool cand = y < n && y != p && g.id_of_slot[y] >= 0 && (uint32_t)wo[y] < (uint32_t)g.nin_beta[y];
        unsigned long long m = __ballot(cand);
        while (m) {  // wave-uniform
            int32_t yq[4];
            take4(m, y0, yq);
            ListRegs r[4];
            uint32_t w[4];
#pragma unroll
            for (int q = 0; q < 4; ++q)
                if (yq[q] >= 0) {
                    r[q] = list_load(g, yq[q]);
                    w[q] = (uint32_t)wo[yq[q]];
                }
#pragma unroll
            for (int q = 0; q < 4; ++q)
                if (yq[q] >= 0) list_insert_regs(g, yq[q], r[q], p, w[q]);
        }
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------
// mask and recompute (removal, edge increase)
// ---------------------------------------------------------------------------

__device__ inline FusedArgs remove_args(const BatchGraph &bg, const BatchItem &it) {
    FusedArgs fa{};
    fa.mode = FUSED_REMOVE;
    fa.k = it.a;
    fa.col1 = bg.colu;
    fa.row1 = bg.rowu;
    fa.row2 = nullptr;
    return fa;
}

__device__ inline FusedArgs increase_args(const DevGraph &g, const BatchGraph &bg) {
    FusedArgs fa{};
    fa.mode = FUSED_INCREASE;
    fa.k = -1;
    fa.col1 = bg.colu;
    fa.col2 = bg.colv;
    fa.row1 = bg.rowv;
    fa.row2 = g.undirected ? bg.rowu : nullptr;
    return fa;
}

// Flags of rows [r0, r1) into the graph's bitmap (8 lanes assemble each
// 32-column word with shuffles) and the row marks.  S1 / S2: the pair test's
// row vectors (LDS stage or global; S2 used only when fa.row2 is set).
// tests(i): the row's pair tests (row_tests over the graph's vectors, or an
// LDS copy of the chunk's rows).
template <int U, class Tests>
__device__ __forceinline__ void detect_rows(const DevGraph &g, const BatchGraph &bg, const FusedArgs &fa, int32_t r0,
                            int32_t r1, const uint32_t *S1, const uint32_t *S2, Tests tests) {
    const int lane = lane_id();
    const int n = g.n_slots;
    const int64_t nwp = (g.P + 31) / 32;
    uint32_t pmask = 0;  // rows of the current piece holding a flag (wave-uniform)
    stream_chunks<U>(
        g, n, r0, r1,
        [&](int32_t i) {
            const RowTests rt = tests(i);
            return rt.t1 || rt.t2;
        },
        [&](int32_t c0) {
            const uint4 v1 = vec4(S1, c0, n);
            return Vec2{v1, fa.row2 ? vec4(S2, c0, n) : v1};
        },
        [&](int32_t i, int32_t c0, bool ok, uint4 d, const Vec2 &v) {
            uint32_t bits = 0;
            if (ok) {
                const RowTests rt = tests(i);
                const uint4 v1 = v.a;
                const uint4 v2 = v.b;
                const uint32_t dv[4] = {d.x, d.y, d.z, d.w};
                const uint32_t w1[4] = {v1.x, v1.y, v1.z, v1.w};
                const uint32_t w2[4] = {v2.x, v2.y, v2.z, v2.w};
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int32_t j = c0 + e;
                    const bool f = j < n && j != i && !(fa.mode == FUSED_REMOVE && j == fa.k) && dv[e] < INF &&
                                   ((rt.t1 && cat(rt.a1, w1[e]) == dv[e]) || (rt.t2 && cat(rt.a2, w2[e]) == dv[e]));
                    bits |= (uint32_t)f << e;
                }
            }
            uint32_t word = bits << ((lane & 7) * 4);
#pragma unroll
            for (int o = 1; o < 8; o <<= 1) word |= (uint32_t)__shfl_xor((int)word, o);
            if (ok && (lane & 7) == 0 && word != 0) bg.flag_bits[(int64_t)i * nwp + (c0 >> 5)] = word;
            if (__ballot(ok && word != 0) != 0) pmask |= 1u << (i & 31);
        },
        [&](int32_t i0) {
            // the U rows of a piece share a word of row marks (r0 is a
            // multiple of 16, U of 4 up to 16): one atomic per piece that
            // has a flag
            if (lane == 0 && pmask) atomicOr(&bg.row_bits[i0 >> 5], pmask);
            pmask = 0;
        });
}

// Bellman-Ford over the flagged columns of row Drow read straight from its
// flag words fw[0..nw) (no list): 16 groups of 4 lanes take words round
// robin, a group relaxes the columns of its word one at a time, 32 index
// entries per round trip, stopping once an entry is at least the current
// value.  Columns left above their index bound are marked in `need` (nw
// words of LDS) and get exhaustive scans by the whole wavefront; the sweeps
// resume if that changed anything.
__device__ __forceinline__ void wave_bellman_ford_words(const DevGraph &g, int32_t *Drow, const uint32_t *fw, int nw,
                                                        uint32_t *need) {
    const int lane = lane_id();
    const int g4 = lane >> 2, l4 = lane & 3;
    const int lim = g.lim;
    const int n = g.n_slots;
    const int32_t *Min = in_matrix(g);
    for (;;) {
        for (;;) {
            bool changed = false;
            for (int w = g4; w < nw; w += 16) {
                uint32_t bits = fw[w];
                while (bits) {
                    const int32_t y = w * 32 + __ffs(bits) - 1;
                    bits &= bits - 1;
                    uint32_t best = (uint32_t)Drow[y];
                    const int4 *L4 = reinterpret_cast<const int4 *>(g.nin + (int64_t)y * NIN_L);
                    for (int c0 = 0; c0 < lim; c0 += 32) {
                        const int e0 = c0 + 4 * l4, e1 = e0 + 16;
                        const int4 none = make_int4(0, (int)INF, 0, (int)INF);
                        int4 pa = none, pb = none, pc = none, pd = none;
                        if (e0 < lim) pa = L4[e0 >> 1];
                        if (e0 + 2 < lim) pb = L4[(e0 >> 1) + 1];
                        if (e1 < lim) pc = L4[e1 >> 1];
                        if (e1 + 2 < lim) pd = L4[(e1 >> 1) + 1];
                        if (e0 + 1 >= lim) pa.w = (int)INF;
                        if (e0 + 3 >= lim) pb.w = (int)INF;
                        if (e1 + 1 >= lim) pc.w = (int)INF;
                        if (e1 + 3 >= lim) pd.w = (int)INF;
                        uint32_t cm = INF;
                        if ((uint32_t)pa.y < best) cm = min(cm, cat((uint32_t)Drow[pa.x], (uint32_t)pa.y));
                        if ((uint32_t)pa.w < best) cm = min(cm, cat((uint32_t)Drow[pa.z], (uint32_t)pa.w));
                        if ((uint32_t)pb.y < best) cm = min(cm, cat((uint32_t)Drow[pb.x], (uint32_t)pb.y));
                        if ((uint32_t)pb.w < best) cm = min(cm, cat((uint32_t)Drow[pb.z], (uint32_t)pb.w));
                        if ((uint32_t)pc.y < best) cm = min(cm, cat((uint32_t)Drow[pc.x], (uint32_t)pc.y));
                        if ((uint32_t)pc.w < best) cm = min(cm, cat((uint32_t)Drow[pc.z], (uint32_t)pc.w));
                        if ((uint32_t)pd.y < best) cm = min(cm, cat((uint32_t)Drow[pd.x], (uint32_t)pd.y));
                        if ((uint32_t)pd.w < best) cm = min(cm, cat((uint32_t)Drow[pd.z], (uint32_t)pd.w));
                        cm = min(cm, (uint32_t)__shfl_xor((int)cm, 1, 4));
                        cm = min(cm, (uint32_t)__shfl_xor((int)cm, 2, 4));
                        best = min(best, cm);
                        const uint32_t wlast = (uint32_t)__shfl(pd.w, 3, 4);
                        if (wlast >= best) break;
                    }
                    if (l4 == 0 && best < (uint32_t)Drow[y]) {
                        Drow[y] = (int32_t)best;
                        changed = true;
                    }
                }
            }
            __threadfence_block();
            if (!__any(changed)) break;
        }
        // columns above their bound -> need (LDS bitmap of this wavefront)
        for (int w = lane; w < nw; w += 64) need[w] = 0;
        __threadfence_block();
        for (int w = g4; w < nw; w += 16) {
            uint32_t bits = fw[w];
            uint32_t mark = 0;
            while (bits) {
                const int b = __ffs(bits) - 1;
                bits &= bits - 1;
                const int32_t y = w * 32 + b;
                uint32_t beta_eff = (uint32_t)g.nin_beta[y];
                if (lim < NIN_L) beta_eff = min(beta_eff, (uint32_t)g.nin[(int64_t)y * NIN_L + lim].y);
                if ((uint32_t)Drow[y] > beta_eff) mark |= 1u << b;
            }
            if (l4 == 0 && mark) need[w] = mark;
        }
        __threadfence_block();
        bool changed = false;
        for (int w = 0; w < nw; ++w) {  // wave-uniform: every lane reads the same LDS word
            uint32_t bits = need[w];
            while (bits) {
                const int32_t y = w * 32 + __ffs(bits) - 1;
                bits &= bits - 1;
                const int32_t *col = Min + (int64_t)y * g.ld;
                const uint32_t best = wave_min_plus(Drow, col, n);
                if (best < (uint32_t)Drow[y]) {
                    changed = true;
                    if (lane == 0) Drow[y] = (int32_t)best;
                }
                __threadfence_block();
            }
        }
        if (!changed) break;
    }
}

// Recompute of the flagged rows among [r0, r1): one wavefront per row, rows
// dealt round robin to the 4 wavefronts.  The row's flagged entries (and
// column k of a removal) start at INF and are relaxed in place; rows with at
// most ROW_CAP flags use a list in LDS (wlists: 2 ROW_CAP words per wave);
// larger ones use a list in global memory (glists: 2 P words per wave) or,
// without one, read their flag words directly (needs: 4 * ceil(P / 32)
// words of LDS).
__device__ __forceinline__ void recompute_rows(const DevGraph &g, const BatchGraph &bg, const FusedArgs &fa, int32_t r0, int32_t r1,
                               int32_t *wlists, int32_t *glists, uint32_t *needs, bool defer_heavy = false,
                               uint32_t *light = nullptr) {
    const int lane = lane_id(), wv = threadIdx.x >> 6;
    const int nw = (g.n_slots + 31) / 32;
    const int64_t nwp = (g.P + 31) / 32;
    int32_t *list = wlists + wv * 2 * ROW_CAP;
    int32_t *fsl = list + ROW_CAP;
    int32_t *glist = glists ? glists + (int64_t)wv * 2 * g.P : nullptr;
    int nfs = 0;
    for (int32_t i = r0 + wv; i < r1; i += BATCH_THREADS / 64) {
        {
            if (((bg.row_bits[i >> 5] >> (i & 31)) & 1u) == 0) continue;
            uint32_t *fw = bg.flag_bits + (int64_t)i * nwp;
            int cnt = 0;
            for (int b = 0; b < nw; b += 512) {  // wave-uniform; 8 words per lane in flight
                uint32_t wd[8];
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    const int w = b + q * 64 + lane;
                    wd[q] = w < nw ? fw[w] : 0u;
                }
                int c = 0;
#pragma unroll
                for (int q = 0; q < 8; ++q) c += __popc(wd[q]);
                int incl = c;
#pragma unroll
                for (int o = 1; o < 64; o <<= 1) {
                    const int t = __shfl_up(incl, o);
                    if (lane >= o) incl += t;
                }
                int pos = cnt + incl - c;
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    uint32_t bits = wd[q];
                    while (bits) {
                        const int bt = __ffs(bits) - 1;
                        bits &= bits - 1;
                        const int32_t col = (b + q * 64 + lane) * 32 + bt;
                        if (pos < ROW_CAP) list[pos] = col;
                        if (glist) glist[pos] = col;
                        ++pos;
                    }
                }
                cnt += __shfl(incl, 63);
            }
            if (defer_heavy && cnt > ROW_CAP) {  // one work-group per row later
                if (lane == 0) bg.heavy_rows[atomicAdd(&g.ctl->heavy_count, 1)] = i;
                continue;
            }
            __threadfence_block();
            int32_t *Drow = g.D + (int64_t)i * g.ld;
            if (light && cnt <= ROW_CAP) {
                // the values stay in LDS: one pull per entry and a closure
                // (light_row); flagged entries of D are neither reset nor read
                const LightRowLds L = light_row_lds(light + wv * LIGHT_ROW_WORDS);
                if (fa.mode == FUSED_REMOVE && lane == 0) Drow[fa.k] = (int32_t)INF;
                __threadfence_block();
                const uint32_t w_old = fa.mode == FUSED_INCREASE ? (uint32_t)g.ctl->w_old : 0u;
                int sweeps = 0;
                const uint32_t v = light_row(g, fa, row_tests(g, fa, i, w_old), Drow, list, cnt, L.fsl, L.old, L.val,
                                             L.keys, L.pos, L.W, sweeps, nfs);
                if (lane < cnt) Drow[list[lane]] = (int32_t)v;
                for (int w = lane; w < nw; w += 64)
                    if (fw[w]) fw[w] = 0u;
                continue;
            }
            if (cnt <= ROW_CAP || glist) {
                const int32_t *L = cnt <= ROW_CAP ? list : glist;
                for (int e = lane; e < cnt; e += 64) Drow[L[e]] = (int32_t)INF;
            } else {
                for (int w = lane; w < nw; w += 64) {
                    uint32_t bits = fw[w];
                    while (bits) {
                        Drow[w * 32 + __ffs(bits) - 1] = (int32_t)INF;
                        bits &= bits - 1;
                    }
                }
            }
            if (fa.mode == FUSED_REMOVE && lane == 0) Drow[fa.k] = (int32_t)INF;
            __threadfence_block();
            int sweeps = 0;
            if (cnt <= ROW_CAP) wave_bellman_ford(g, Drow, list, cnt, fsl, sweeps, nfs);
            else if (glist) wave_bellman_ford(g, Drow, glist, cnt, glist + g.P, sweeps, nfs);
            else wave_bellman_ford_words(g, Drow, fw, nw, needs + wv * ((g.P + 31) / 32));
            // the row's flag words are used up: leave the bitmap clear
            for (int w = lane; w < nw; w += 64)
                if (fw[w]) fw[w] = 0u;
        }
    }
}

__device__ inline void clear_row_marks(const DevGraph &g, const BatchGraph &bg) {
    for (int w = threadIdx.x; w < (g.n_slots + 31) / 32; w += BATCH_THREADS) bg.row_bits[w] = 0;
}

// Rebuild the index lists of y when they have shrunk (block-wide select).
__device__ __forceinline__ void batch_rebuild_if_short(const DevGraph &g, int32_t y, SelectShared &ssh, uint32_t *stage) {
    if (!(g.nin_cnt[y] < NIN_L / 2 && (uint32_t)g.nin_beta[y] < INF && g.id_of_slot[y] >= 0)) return;
    select_light(in_matrix(g) + (int64_t)y * g.ld, g.n_slots, y, g.nin + (int64_t)y * NIN_L, g.nin_cnt + y,
                 g.nin_beta + y, ssh, stage);
}

__device__ __forceinline__ void remove_prologue(const DevGraph &g, const BatchGraph &bg, const BatchItem &it) {
    const int32_t k = it.a;
    if (threadIdx.x == 0) g.ctl->heavy_count = 0;
    for (int32_t i = threadIdx.x; i < g.n_slots; i += BATCH_THREADS) {
        bg.colu[i] = g.D[(int64_t)i * g.ld + k];
        bg.rowu[i] = g.D[(int64_t)k * g.ld + i];
    }
    __syncthreads();
}

// Row marks cleared, k dropped from every index list, tombstone, short lists
// rebuilt, ranks shifted.
__device__ __forceinline__ void remove_epilogue(const DevGraph &g, const BatchGraph &bg, const BatchItem &it, SelectShared &ssh,
                                uint32_t *stage) {
    const int tid = threadIdx.x;
    const int n = g.n_slots;
    const int32_t k = it.a, rank = it.b, n_live = it.c;
    clear_row_marks(g, bg);
    // lanes screen 64 lists at a time: k can be listed in y only if its edge
    // is no heavier than y's last entry
    for (int32_t y0 = (tid >> 6) * 64; y0 < n; y0 += BATCH_THREADS) {
        const int32_t y = y0 + lane_id();
        bool cand = false;
        if (y < n && y != k) {
            const int c = g.nin_cnt[y];
            const uint32_t wk = (uint32_t)g.A[(int64_t)k * g.ld + y];
            cand = c > 0 && wk < INF && wk <= (uint32_t)g.nin[(int64_t)y * NIN_L + c - 1].y;
        }
        unsigned long long m = __ballot(cand);
        while (m) {  // wave-uniform
            int32_t yq[4];
            take4(m, y0, yq);
            ListRegs r[4];
#pragma unroll
            for (int q = 0; q < 4; ++q)
                if (yq[q] >= 0) r[q] = list_load(g, yq[q]);
#pragma unroll
            for (int q = 0; q < 4; ++q)
                if (yq[q] >= 0) list_purge_regs(g, yq[q], r[q], k);
        }
    }
    if (tid < 64) {
        g.nin[(int64_t)k * NIN_L + tid] = make_int2(0, (int)INF);
        if (tid == 0) {
            g.nin_cnt[k] = 0;
            g.nin_beta[k] = (int32_t)INF;
        }
    }
    __syncthreads();
    const int64_t ld = g.ld;
    for (int32_t s = tid; s < n; s += BATCH_THREADS) {
        g.D[(int64_t)k * ld + s] = (int32_t)INF;
        g.D[(int64_t)s * ld + k] = (int32_t)INF;
        g.A[(int64_t)k * ld + s] = (int32_t)INF;
        g.A[(int64_t)s * ld + k] = (int32_t)INF;
        if (!g.undirected) {
            g.AT[(int64_t)k * ld + s] = (int32_t)INF;
            g.AT[(int64_t)s * ld + k] = (int32_t)INF;
        }
    }
    if (tid == 0) g.id_of_slot[k] = -1;
    __syncthreads();
    // rebuild the lists that fell below half (rare)
    __shared__ int32_t s_cnt;
    if (tid == 0) s_cnt = 0;
    __syncthreads();
    for (int32_t y = tid; y < n; y += BATCH_THREADS)
        if (g.nin_cnt[y] < NIN_L / 2 && (uint32_t)g.nin_beta[y] < INF && g.id_of_slot[y] >= 0)
            bg.queue[atomicAdd(&s_cnt, 1)] = y;
    __syncthreads();
    const int nq = s_cnt;
    for (int q = 0; q < nq; ++q) batch_rebuild_if_short(g, bg.queue[q], ssh, stage);
    for (int32_t t = tid; t < n_live - 1; t += BATCH_THREADS) it.rank_dst[t] = it.rank_src[t < rank ? t : t + 1];
    __syncthreads();
}

// ---------------------------------------------------------------------------
// edge update
// ---------------------------------------------------------------------------

// The decision (decrease / increase / nothing, on the device), the new
// weight in A and the index lists, and the gathers the sweeps need.
__device__ __forceinline__ void edge_prologue(const DevGraph &g, const BatchGraph &bg, const BatchItem &it) {
    const int32_t su = it.a, sv = it.b, w = it.c;
    if (threadIdx.x < 64) edge_begin_wave(g, su, sv, w);
    __syncthreads();
    if (g.ctl->edge_mode != EDGE_NOOP) {
        for (int32_t i = threadIdx.x; i < g.n_slots; i += BATCH_THREADS) {
            bg.colu[i] = g.D[(int64_t)i * g.ld + su];
            bg.colv[i] = g.D[(int64_t)i * g.ld + sv];
            bg.rowu[i] = g.D[(int64_t)su * g.ld + i];
            bg.rowv[i] = g.D[(int64_t)sv * g.ld + i];
        }
    }
    __syncthreads();
}

// Relaxation through the lowered edge over rows [r0, r1): D[i][j] vs
// D[i][u] (+) w (+) D[v][j] (and D[i][v] (+) w (+) D[u][j] when undirected), rows
// that cannot change filtered first.  SV / SU: rows v and u (LDS or global).
// cu(i), cv(i): D[i][u] and D[i][v] (the graph's vectors or an LDS copy of
// the chunk's rows).
template <int U, class ColU, class ColV>
__device__ __forceinline__ void dec_relax_rows(const DevGraph &g, const BatchGraph &bg, int32_t w, int32_t r0, int32_t r1,
                               const uint32_t *SV, const uint32_t *SU, ColU cu, ColV cv) {
    const bool und = g.undirected != 0;
    const uint32_t wn = (uint32_t)w;
    const int n = g.n_slots;
    stream_chunks<U>(
        g, n, r0, r1,
        [&](int32_t i) {
            const uint32_t du = cu(i), dv = cv(i);
            return cat(du, wn) < dv || (und && cat(dv, wn) < du);
        },
        [&](int32_t c0) {
            return Vec2{vec4(SV, c0, n), und ? vec4(SU, c0, n) : make_uint4(INF, INF, INF, INF)};
        },
        [&](int32_t i, int32_t c0, bool ok, uint4 d, const Vec2 &v) {
            if (!ok) return;
            const uint32_t du = cu(i), dv = cv(i);
            const uint32_t x1 = cat(du, wn) < dv ? cat(du, wn) : INF;
            const uint32_t x2 = und && cat(dv, wn) < du ? cat(dv, wn) : INF;
            const uint4 rv = v.a;
            const uint4 ru = v.b;
            store_min4(g, i, c0, d,
                       make_uint4(min(cat(x1, rv.x), cat(x2, ru.x)), min(cat(x1, rv.y), cat(x2, ru.y)),
                                  min(cat(x1, rv.z), cat(x2, ru.z)), min(cat(x1, rv.w), cat(x2, ru.w))));
        });
}

__device__ __forceinline__ void edge_epilogue(const DevGraph &g, const BatchGraph &bg, const BatchItem &it, SelectShared &ssh,
                              uint32_t *stage) {
    if (g.ctl->edge_mode == EDGE_INCREASE) clear_row_marks(g, bg);
    batch_rebuild_if_short(g, it.b, ssh, stage);
    if (g.undirected) batch_rebuild_if_short(g, it.a, ssh, stage);
    __syncthreads();
}

// One heavy row with the whole work-group: row i of D in LDS (cur, P words),
// its flagged entries (from the flag words) set to INF (and column k of a
// removal), Bellman-Ford with 64 groups of 4 lanes reading cur from LDS,
// exhaustive scans (marked in need: nw LDS words) by the whole work-group,
// then the flagged entries written back.
__device__ __forceinline__ void heavy_row_block(const DevGraph &g, const BatchGraph &bg, const FusedArgs &fa, int32_t i,
                                                uint32_t *cur, uint32_t *need, int *s_flag, uint32_t *red) {
    const int tid = threadIdx.x, grp = tid >> 2, l4 = tid & 3;
    const int n = g.n_slots;
    const int nw = (n + 31) / 32;
    const int64_t nwp = (g.P + 31) / 32;
    const int lim = g.lim;
    const int32_t *Min = in_matrix(g);
    int32_t *Drow = g.D + (int64_t)i * g.ld;
    uint32_t *fw = bg.flag_bits + (int64_t)i * nwp;
    for (int32_t c = tid * 4; c < n; c += BATCH_THREADS * 4)
        *reinterpret_cast<uint4 *>(cur + c) = *reinterpret_cast<const uint4 *>(Drow + c);
    __syncthreads();
    for (int w = tid; w < nw; w += BATCH_THREADS) {
        uint32_t bits = fw[w];
        while (bits) {
            cur[w * 32 + __ffs(bits) - 1] = INF;
            bits &= bits - 1;
        }
    }
    if (fa.mode == FUSED_REMOVE && tid == 0) cur[fa.k] = INF;
    for (;;) {
        for (;;) {
            __syncthreads();
            if (tid == 0) *s_flag = 0;
            __syncthreads();
            bool changed = false;
            // a group takes 8 columns (a quarter of a flag word) at a time, so
            // that a dense word is shared by four groups
            for (int u = grp; u < 4 * nw; u += BATCH_THREADS / 4) {
                uint32_t bits = (fw[u >> 2] >> (8 * (u & 3))) & 0xFFu;
                while (bits) {
                    const int32_t y = (u >> 2) * 32 + 8 * (u & 3) + __ffs(bits) - 1;
                    bits &= bits - 1;
                    uint32_t best = cur[y];
                    const int4 *L4 = reinterpret_cast<const int4 *>(g.nin + (int64_t)y * NIN_L);
                    for (int c0 = 0; c0 < lim; c0 += 32) {
                        const int e0 = c0 + 4 * l4, e1 = e0 + 16;
                        const int4 none = make_int4(0, (int)INF, 0, (int)INF);
                        int4 pa = none, pb = none, pc = none, pd = none;
                        if (e0 < lim) pa = L4[e0 >> 1];
                        if (e0 + 2 < lim) pb = L4[(e0 >> 1) + 1];
                        if (e1 < lim) pc = L4[e1 >> 1];
                        if (e1 + 2 < lim) pd = L4[(e1 >> 1) + 1];
                        if (e0 + 1 >= lim) pa.w = (int)INF;
                        if (e0 + 3 >= lim) pb.w = (int)INF;
                        if (e1 + 1 >= lim) pc.w = (int)INF;
                        if (e1 + 3 >= lim) pd.w = (int)INF;
                        uint32_t cm = INF;
                        if ((uint32_t)pa.y < best) cm = min(cm, cat(cur[pa.x], (uint32_t)pa.y));
                        if ((uint32_t)pa.w < best) cm = min(cm, cat(cur[pa.z], (uint32_t)pa.w));
                        if ((uint32_t)pb.y < best) cm = min(cm, cat(cur[pb.x], (uint32_t)pb.y));
                        if ((uint32_t)pb.w < best) cm = min(cm, cat(cur[pb.z], (uint32_t)pb.w));
                        if ((uint32_t)pc.y < best) cm = min(cm, cat(cur[pc.x], (uint32_t)pc.y));
                        if ((uint32_t)pc.w < best) cm = min(cm, cat(cur[pc.z], (uint32_t)pc.w));
                        if ((uint32_t)pd.y < best) cm = min(cm, cat(cur[pd.x], (uint32_t)pd.y));
                        if ((uint32_t)pd.w < best) cm = min(cm, cat(cur[pd.z], (uint32_t)pd.w));
                        cm = min(cm, (uint32_t)__shfl_xor((int)cm, 1, 4));
                        cm = min(cm, (uint32_t)__shfl_xor((int)cm, 2, 4));
                        best = min(best, cm);
                        const uint32_t wlast = (uint32_t)__shfl(pd.w, 3, 4);
                        if (wlast >= best) break;
                    }
                    if (l4 == 0 && best < cur[y]) {
                        cur[y] = best;
                        changed = true;
                    }
                }
            }
            if (changed) *s_flag = 1;
            __syncthreads();
            if (*s_flag == 0) break;
        }
        for (int w = tid; w < nw; w += BATCH_THREADS) need[w] = 0;
        __syncthreads();
        for (int u = grp; u < 4 * nw; u += BATCH_THREADS / 4) {  // quarter words, as in the sweeps
            const int sh8 = 8 * (u & 3);
            uint32_t bits = (fw[u >> 2] >> sh8) & 0xFFu, mark = 0;
            while (bits) {
                const int b = __ffs(bits) - 1;
                bits &= bits - 1;
                const int32_t y = (u >> 2) * 32 + sh8 + b;
                uint32_t beta_eff = (uint32_t)g.nin_beta[y];
                if (lim < NIN_L) beta_eff = min(beta_eff, (uint32_t)g.nin[(int64_t)y * NIN_L + lim].y);
                if (cur[y] > beta_eff) mark |= 1u << (sh8 + b);
            }
            if (l4 == 0 && mark) atomicOr(&need[u >> 2], mark);
        }
        __syncthreads();
        if (tid == 0) *s_flag = 0;
        for (int w = 0; w < nw; ++w) {  // block-uniform: every thread reads the same LDS word
            uint32_t bits = need[w];
            while (bits) {
                const int32_t y = w * 32 + __ffs(bits) - 1;
                bits &= bits - 1;
                const int32_t *col = Min + (int64_t)y * g.ld;
                uint32_t best = INF;
                for (int32_t x = tid; x < n; x += BATCH_THREADS) best = min(best, cat(cur[x], (uint32_t)col[x]));
                best = block_min<BATCH_THREADS>(best, red);
                if (tid == 0 && best < cur[y]) {
                    cur[y] = best;
                    *s_flag = 1;
                }
                __syncthreads();
            }
        }
        __syncthreads();
        if (*s_flag == 0) break;
    }
    for (int w = tid; w < nw; w += BATCH_THREADS) {
        uint32_t bits = fw[w];
        if (bits) fw[w] = 0u;  // used up: the bitmap is left clear
        while (bits) {
            const int32_t y = w * 32 + __ffs(bits) - 1;
            bits &= bits - 1;
            Drow[y] = (int32_t)cur[y];
        }
    }
    __syncthreads();
}

// heavy_row_block with the row's flagged columns compacted once into an LDS
// list (`list`: room for n entries): the sweeps hand out entries, not flag
// words, so a dense word does not become one group's chain, and each group
// keeps its first entry's 32 lightest in-edges in registers across the
// sweeps.  Same fixed point, same writes.
__device__ __forceinline__ void heavy_row_block_listed(const DevGraph &g, const BatchGraph &bg, const FusedArgs &fa,
                                                       int32_t i, uint32_t *cur, int32_t *list, uint32_t *need,
                                                       int *s_flag, uint32_t *red) {
    const int tid = threadIdx.x, grp = tid >> 2, l4 = tid & 3;
    constexpr int NG = BATCH_THREADS / 4;
    const int n = g.n_slots;
    const int nw = (n + 31) / 32;
    const int64_t nwp = (g.P + 31) / 32;
    const int lim = g.lim;
    const int32_t *Min = in_matrix(g);
    int32_t *Drow = g.D + (int64_t)i * g.ld;
    uint32_t *fw = bg.flag_bits + (int64_t)i * nwp;
    for (int32_t c = tid * 4; c < n; c += BATCH_THREADS * 4)
        *reinterpret_cast<uint4 *>(cur + c) = *reinterpret_cast<const uint4 *>(Drow + c);
    // compact the flagged columns: a thread per word, then a block scan
    int total = 0;
    for (int w0 = 0; w0 < nw; w0 += BATCH_THREADS) {
        const int w = w0 + tid;
        const uint32_t bits0 = w < nw ? fw[w] : 0u;
        int tot;
        int pos = total + block_exscan<BATCH_THREADS>(__popc(bits0), red, &tot);
        for (uint32_t bits = bits0; bits; bits &= bits - 1) list[pos++] = w * 32 + __ffs(bits) - 1;
        total += tot;
        __syncthreads();
    }
    for (int e = tid; e < total; e += BATCH_THREADS) cur[list[e]] = INF;
    if (fa.mode == FUSED_REMOVE && tid == 0) cur[fa.k] = INF;
    __syncthreads();
    const bool has0 = grp < total;
    const int32_t y0 = has0 ? list[grp] : 0;
    const int4 *Y4 = reinterpret_cast<const int4 *>(g.nin + (int64_t)y0 * NIN_L);
    const int4 none4 = make_int4(0, (int)INF, 0, (int)INF);
    const int4 q0 = has0 ? index_pair(Y4, lim, 2 * l4) : none4, q1 = has0 ? index_pair(Y4, lim, 8 + 2 * l4) : none4;
    const int4 q2 = has0 ? index_pair(Y4, lim, 16 + 2 * l4) : none4, q3 = has0 ? index_pair(Y4, lim, 24 + 2 * l4) : none4;
    const uint32_t wl0 = (uint32_t)__shfl(q3.w, 3, 4);  // entry 31 (INF past lim)
    for (;;) {
        for (;;) {
            __syncthreads();
            if (tid == 0) *s_flag = 0;
            __syncthreads();
            bool changed = false;
            for (int e = grp; e < total; e += NG) {
                const int32_t y = e == grp ? y0 : list[e];
                const int4 *L4 = reinterpret_cast<const int4 *>(g.nin + (int64_t)y * NIN_L);
                uint32_t best = cur[y];
                uint32_t cm;
                uint32_t wl;
                if (e == grp) {
                    cm = pull_pair(cur, q0, best, INF);
                    cm = pull_pair(cur, q1, best, cm);
                    cm = pull_pair(cur, q2, best, cm);
                    cm = pull_pair(cur, q3, best, cm);
                    wl = wl0;
                } else {
                    const int4 r0 = index_pair(L4, lim, 2 * l4), r1 = index_pair(L4, lim, 8 + 2 * l4);
                    const int4 r2 = index_pair(L4, lim, 16 + 2 * l4), r3 = index_pair(L4, lim, 24 + 2 * l4);
                    cm = pull_pair(cur, r0, best, INF);
                    cm = pull_pair(cur, r1, best, cm);
                    cm = pull_pair(cur, r2, best, cm);
                    cm = pull_pair(cur, r3, best, cm);
                    wl = (uint32_t)__shfl(r3.w, 3, 4);
                }
                best = min(best, group4_min(cm));
                for (int c0 = 32; c0 < lim && wl < best; c0 += 32) {  // rare: the rest of the list
                    uint32_t cr = INF;
#pragma unroll
                    for (int q = 0; q < 4; ++q) cr = pull_pair(cur, index_pair(L4, lim, c0 + 8 * q + 2 * l4), best, cr);
                    best = min(best, group4_min(cr));
                    wl = (uint32_t)__shfl(index_pair(L4, lim, c0 + 24 + 2 * l4).w, 3, 4);
                }
                if (l4 == 0 && best < cur[y]) {
                    cur[y] = best;
                    changed = true;
                }
            }
            if (changed) *s_flag = 1;
            __syncthreads();
            if (*s_flag == 0) break;
        }
        for (int w = tid; w < nw; w += BATCH_THREADS) need[w] = 0;
        __syncthreads();
        for (int e = tid; e < total; e += BATCH_THREADS) {
            const int32_t y = list[e];
            uint32_t beta_eff = (uint32_t)g.nin_beta[y];
            if (lim < NIN_L) beta_eff = min(beta_eff, (uint32_t)g.nin[(int64_t)y * NIN_L + lim].y);
            if (cur[y] > beta_eff) atomicOr(&need[y >> 5], 1u << (y & 31));
        }
        __syncthreads();
        if (tid == 0) *s_flag = 0;
        for (int w = 0; w < nw; ++w) {  // block-uniform: every thread reads the same LDS word
            uint32_t bits = need[w];
            while (bits) {
                const int32_t y = w * 32 + __ffs(bits) - 1;
                bits &= bits - 1;
                const int32_t *col = Min + (int64_t)y * g.ld;
                uint32_t best = INF;
                for (int32_t x = tid; x < n; x += BATCH_THREADS) best = min(best, cat(cur[x], (uint32_t)col[x]));
                best = block_min<BATCH_THREADS>(best, red);
                if (tid == 0 && best < cur[y]) {
                    cur[y] = best;
                    *s_flag = 1;
                }
                __syncthreads();
            }
        }
        __syncthreads();
        if (*s_flag == 0) break;
    }
    for (int e = tid; e < total; e += BATCH_THREADS) {
        const int32_t y = list[e];
        Drow[y] = (int32_t)cur[y];
    }
    for (int w = tid; w < nw; w += BATCH_THREADS)
        if (fw[w]) fw[w] = 0u;  // used up: the bitmap is left clear
    __syncthreads();
}

// Algorithm 7's query; a widest graph's distance goes out as a width.
__device__ __forceinline__ void batch_query(const DevGraph &g, const BatchGraph &bg, const BatchItem &it) {
    query_block(g, it.a, it.b, it.out, bg.qscratch);
    if (g.widest && threadIdx.x == 0) it.out[0] = widest_xf(it.out[0]);  // the thread that wrote it
    __syncthreads();
}

// ---------------------------------------------------------------------------
// schedule 1: work queue (one work-group per graph, all phases)
// ---------------------------------------------------------------------------

template <int U>
__device__ __forceinline__ void run_item_alone(const DevGraph &g, const BatchGraph &bg, const BatchItem &it, SelectShared &ssh,
                               uint32_t *stage, int32_t *wlists) {
    const int n = g.n_slots;
    switch (it.op) {
    case BOP_ADD:
        add_prologue(g, bg, it, ssh, stage);
        stage_rows(stage, g.P, n, bg.vout, nullptr);
        add_relax_rows<U>(g, bg, 0, n, stage, [&](int32_t i) { return (uint32_t)(g.undirected ? bg.vout : bg.vin)[i]; });
        __syncthreads();
        add_epilogue(g, bg, it);
        break;
    case BOP_REMOVE: {
        remove_prologue(g, bg, it);
        const FusedArgs fa = remove_args(bg, it);
        stage_rows(stage, g.P, n, fa.row1, nullptr);
        detect_rows<U>(g, bg, fa, 0, n, stage, stage + g.P, [&](int32_t i) { return row_tests(g, fa, i, 0u); });
        __syncthreads();
        recompute_rows(g, bg, fa, 0, n, wlists, bg.scratch, stage);
        __syncthreads();
        remove_epilogue(g, bg, it, ssh, stage);
        break;
    }
    case BOP_EDGE: {
        edge_prologue(g, bg, it);
        const int32_t mode = g.ctl->edge_mode;
        if (mode == EDGE_DECREASE) {
            stage_rows(stage, g.P, n, bg.rowv, g.undirected ? bg.rowu : nullptr);
            dec_relax_rows<U>(g, bg, it.c, 0, n, stage, stage + g.P, [&](int32_t i) { return (uint32_t)bg.colu[i]; },
                              [&](int32_t i) { return (uint32_t)bg.colv[i]; });
            __syncthreads();
        } else if (mode == EDGE_INCREASE) {
            const FusedArgs fa = increase_args(g, bg);
            stage_rows(stage, g.P, n, fa.row1, fa.row2);
            const uint32_t w_old = (uint32_t)g.ctl->w_old;
            detect_rows<U>(g, bg, fa, 0, n, stage, stage + g.P, [&](int32_t i) { return row_tests(g, fa, i, w_old); });
            __syncthreads();
            recompute_rows(g, bg, fa, 0, n, wlists, bg.scratch, stage);
            __syncthreads();
        }
        edge_epilogue(g, bg, it, ssh, stage);
        break;
    }
    case BOP_QUERY: batch_query(g, bg, it); break;
    default: break;
    }
    __syncthreads();
}

template <int U>
__global__ __launch_bounds__(BATCH_THREADS, 2) void k_batch(BatchHeader *hdr, const BatchGraph *graphs,
                                                            const int32_t *order, const BatchItem *items) {
    extern __shared__ __align__(16) uint32_t stage[];  // 2 P words of row vectors / select staging, then 4 wave lists of 2 ROW_CAP
    __shared__ SelectShared ssh;
    __shared__ int32_t s_next;
    const int32_t num_graphs = hdr->num_graphs;
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) s_next = atomicAdd(&hdr->counter, 1);
        __syncthreads();
        const int32_t idx = s_next;
        if (idx >= num_graphs) break;
        const BatchGraph &bg = graphs[order[idx]];
        int32_t *wlists = reinterpret_cast<int32_t *>(stage) + 2 * bg.g.P;
        if (threadIdx.x == 0) hdr->times[2 * bg.index] = wall_clock64();
        for (int32_t t = bg.item_begin; t < bg.item_end; ++t) {
            const BatchItem it = items[t];
            DevGraph g = bg.g;
            g.n_slots = it.n_slots;
            run_item_alone<U>(g, bg, it, ssh, stage, wlists);
        }
        if (threadIdx.x == 0) hdr->times[2 * bg.index + 1] = wall_clock64();
    }
}

// ---------------------------------------------------------------------------
// schedule 2: lockstep (whole grid on every step's row sweeps)
// ---------------------------------------------------------------------------

constexpr long BARRIER_SPIN_LIMIT = 1L << 21;  // about a second of polling, then a reported timeout

// Grid barrier in two levels (8 groups of work-groups, then the groups), with
// release/acquire ordering at device scope.  Every wait is bounded: a timeout
// sets hdr->err and lets the work-group go on, so the launch always ends.
__device__ __forceinline__ void grid_barrier(BatchHeader *hdr) {
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned nb = gridDim.x;
        const unsigned grp = blockIdx.x & 7u;
        const unsigned ngroups = nb < 8 ? nb : 8;
        const unsigned gsize = nb / 8 + (grp < nb % 8 ? 1u : 0u);
        // one release per work-group (its writes, in L2 after the block
        // barrier, written back for the other XCDs) and one acquire on the
        // way out: each device-scope fence costs an L2 walk, and a barrier
        // with four of them per work-group cost ~40 us more
        const unsigned gen = __hip_atomic_load(&hdr->bar_gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const unsigned a = __hip_atomic_fetch_add(&hdr->bar_group[grp * 32], 1u, __ATOMIC_RELEASE,
                                                  __HIP_MEMORY_SCOPE_AGENT);
        if (a == gsize - 1) {
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");  // the group's releases, before passing them on
            __hip_atomic_store(&hdr->bar_group[grp * 32], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const unsigned b = __hip_atomic_fetch_add(&hdr->bar_count, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
            if (b == ngroups - 1) {
                __hip_atomic_store(&hdr->bar_count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_fetch_add(&hdr->bar_gen, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
        // poll with relaxed loads (an acquire per poll would invalidate the
        // caches the still-working work-groups rely on), then one acquire
        long it = 0;
        while (__hip_atomic_load(&hdr->bar_gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == gen &&
               it < BARRIER_SPIN_LIMIT) {
            __builtin_amdgcn_s_sleep(2);
            ++it;
        }
        if (it >= BARRIER_SPIN_LIMIT) atomicOr(&hdr->err, 1);
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    __syncthreads();
}

// Chunk c of a step's sweep table -> graph (base: prefix of chunk counts).
// lo: a graph at or before the answer (the previous chunk's graph: a
// work-group's chunks only move forward); the search gallops from there.
__device__ inline int32_t chunk_graph(const int32_t *base, int32_t num_graphs, int32_t c, int32_t lo = 0) {
    int32_t hi = lo + 1, step = 1;  // base[lo] <= c
    while (hi < num_graphs && base[hi] <= c) {
        lo = hi;
        step <<= 1;
        hi = min(num_graphs, lo + step);
    }
    while (hi - lo > 1) {
        const int32_t mid = (lo + hi) >> 1;
        if (base[mid] <= c) lo = mid;
        else hi = mid;
    }
    return lo;
}

// One chunk of step s's row sweeps: rows [cg * rpc, (cg + 1) * rpc) of
// graph bg's item s (rpc = batch_rows_per_chunk).  The caller separates
// chunks with a block barrier, so the staging area is free on entry.
template <int U>
__device__ inline void sweep_chunk(const BatchGraph &bg, const BatchItem *items, int32_t s, int32_t cg, bool staged,
                                   int32_t P_max, uint32_t *stage) {
    const BatchItem it = items[bg.item_begin + s];
    DevGraph g = bg.g;
    g.n_slots = it.n_slots;
    const int32_t rpc = batch_rows_per_chunk(it.n_slots);
    const int32_t r0 = cg * rpc, r1 = min(r0 + rpc, it.n_slots);
    const int32_t mode = it.op == BOP_EDGE ? g.ctl->edge_mode : EDGE_NOOP;
    // the chunk's inputs besides D: one or two row vectors (the
    // columns' side of the pair test or relaxation) and one or two
    // values per row (its side); with `staged`, copied to LDS once
    // per chunk so that a wavefront's pieces wait only for D
    const int32_t *vsrc1 = nullptr, *vsrc2 = nullptr, *rsrc1 = nullptr, *rsrc2 = nullptr;
    if (it.op == BOP_ADD) {
        vsrc1 = bg.vout;
        rsrc1 = g.undirected ? bg.vout : bg.vin;
    } else if (it.op == BOP_REMOVE) {
        vsrc1 = bg.rowu;
        rsrc1 = bg.colu;
    } else if (mode == EDGE_DECREASE || mode == EDGE_INCREASE) {
        vsrc1 = bg.rowv;
        vsrc2 = g.undirected ? bg.rowu : nullptr;
        rsrc1 = bg.colu;
        rsrc2 = bg.colv;
    } else {
        return;  // block-uniform: a no-op edge update or a query sweeps nothing
    }
    const uint32_t *S1 = reinterpret_cast<const uint32_t *>(vsrc1);
    const uint32_t *S2 = reinterpret_cast<const uint32_t *>(vsrc2);
    const uint32_t *T1 = reinterpret_cast<const uint32_t *>(rsrc1) + r0;
    const uint32_t *T2 = reinterpret_cast<const uint32_t *>(rsrc2 ? rsrc2 + r0 : nullptr);
    if (staged) {
        uint32_t *v1 = stage, *v2 = stage + P_max, *t1 = stage + 2 * P_max, *t2 = t1 + LOCKSTEP_STAGE_ROWS;
        const int32_t n4 = (it.n_slots + 3) & ~3;
        for (int32_t x = threadIdx.x; x < n4; x += BATCH_THREADS) {
            v1[x] = x < it.n_slots ? (uint32_t)vsrc1[x] : INF;
            if (vsrc2) v2[x] = x < it.n_slots ? (uint32_t)vsrc2[x] : INF;
        }
        if (it.op == BOP_ADD && !g.undirected) {
            // a directed add's new column is computed here, for the chunk's
            // rows, instead of in the add-vector phase: it reads the same
            // rows' old values that the relaxation then streams
            add_in_rows(g, bg, it, r0, r1, t1);
        } else {
            for (int32_t r = threadIdx.x; r < r1 - r0; r += BATCH_THREADS) {
                t1[r] = (uint32_t)rsrc1[r0 + r];
                if (rsrc2) t2[r] = (uint32_t)rsrc2[r0 + r];
            }
        }
        __syncthreads();
        S1 = v1;
        S2 = vsrc2 ? v2 : nullptr;
        T1 = t1;
        T2 = rsrc2 ? t2 : nullptr;
    }
    if (it.op == BOP_ADD) {
        add_relax_rows<U>(g, bg, r0, r1, S1, [&](int32_t i) { return T1[i - r0]; });
    } else if (it.op == BOP_REMOVE) {
        const FusedArgs fa = remove_args(bg, it);
        const int32_t k = it.a;
        detect_rows<U>(g, bg, fa, r0, r1, S1, nullptr, [&](int32_t i) {
            const uint32_t dik = T1[i - r0];
            return RowTests{i != k && dik < INF, false, dik, 0u};
        });
    } else if (mode == EDGE_DECREASE) {
        dec_relax_rows<U>(g, bg, it.c, r0, r1, S1, S2, [&](int32_t i) { return T1[i - r0]; },
                          [&](int32_t i) { return T2[i - r0]; });
    } else {
        const FusedArgs fa = increase_args(g, bg);
        const uint32_t w_old = (uint32_t)g.ctl->w_old;
        const bool und = g.undirected != 0;
        detect_rows<U>(g, bg, fa, r0, r1, S1, S2, [&](int32_t i) {
            // the pair tests of row_tests for an increase, from the copies
            const uint32_t cu = T1[i - r0], cv = T2[i - r0];
            RowTests r{cv < INF && cat(cu, w_old) == cv, false, cv, 0u};
            if (und) {
                r.t2 = cu < INF && cat(cv, w_old) == cu;
                r.a2 = cu;
            }
            return r;
        });
    }
}

template <int U>
__global__ __launch_bounds__(BATCH_THREADS, 3) void k_batch_lockstep(BatchHeader *hdr, const BatchGraph *graphs,
                                                                     const BatchItem *items, const int32_t *tables) {
    extern __shared__ __align__(16) uint32_t stage[];  // P words of select staging, then the wave lists / need bitmap
    __shared__ SelectShared ssh;
    __shared__ int32_t s_claim, s_found_g, s_found_j, s_sweep;
    __shared__ int s_flag;
    const int32_t G = hdr->num_graphs;
    const int32_t steps = hdr->steps;
    const int32_t P_max = hdr->p_max;
    int32_t *wlists = reinterpret_cast<int32_t *>(stage) + P_max;
    for (int32_t s = 0; s <= steps; ++s) {
        // A: per graph, the epilogue of item s-1 and the prologue of item s
        for (int32_t gi = blockIdx.x; gi < G; gi += gridDim.x) {
            const BatchGraph &bg = graphs[gi];
            if (s == 0 && threadIdx.x == 0) hdr->times[2 * bg.index] = wall_clock64();
            const int32_t cnt = bg.item_end - bg.item_begin;
            if (s >= 1 && s - 1 < cnt) {
                const BatchItem it = items[bg.item_begin + s - 1];
                DevGraph g = bg.g;
                g.n_slots = it.n_slots;
                if (it.op == BOP_ADD) add_epilogue(g, bg, it);
                else if (it.op == BOP_REMOVE) remove_epilogue(g, bg, it, ssh, stage);
                else if (it.op == BOP_EDGE) edge_epilogue(g, bg, it, ssh, stage);
                if (s == cnt && threadIdx.x == 0) hdr->times[2 * bg.index + 1] = wall_clock64();
            }
            if (s < cnt) {
                const BatchItem it = items[bg.item_begin + s];
                DevGraph g = bg.g;
                g.n_slots = it.n_slots;
                if (it.op == BOP_ADD) add_setup(g, bg, it, ssh, stage);
                else if (it.op == BOP_REMOVE) remove_prologue(g, bg, it);
                else if (it.op == BOP_EDGE) edge_prologue(g, bg, it);
                else if (it.op == BOP_QUERY) batch_query(g, bg, it);
                if (s == cnt - 1 && it.op == BOP_QUERY && threadIdx.x == 0)
                    hdr->times[2 * bg.index + 1] = wall_clock64();
            }
            __syncthreads();
        }
        if (s == steps) break;
        grid_barrier(hdr);
        // A2: the new row and column of every added node, spread over the grid
        const int32_t *baseA2 = tables + (int64_t)s * BATCH_TABLES * (G + 1);
        if (baseA2[G] > 0) {
            for (int32_t c = blockIdx.x, gi = 0; c < baseA2[G]; c += gridDim.x) {
                gi = chunk_graph(baseA2, G, c, gi);
                const BatchGraph &bg = graphs[gi];
                const BatchItem it = items[bg.item_begin + s];
                DevGraph g = bg.g;
                g.n_slots = it.n_slots;
                add_vec_chunk(g, bg, it, c - baseA2[gi]);
                __syncthreads();
            }
            grid_barrier(hdr);
        }
        if (blockIdx.x == 0 && threadIdx.x == 0 && 3 * s < BATCH_PHASE_STAMPS) hdr->phase_ts[3 * s] = wall_clock64();
        // B: row sweeps (relaxation or mask) of every graph.  Chunks are
        // claimed from a counter (the next claim is in flight while the
        // current chunk streams), in the table's order: additions and
        // removals first, largest graph first, then the edge updates, most of
        // which turn out to sweep nothing (decided in phase A), so they fill
        // the tail.  A static round robin left the busiest work-group about
        // twice the mean bytes.
        const int32_t *baseB = baseA2 + (G + 1);
        const int32_t *orderB = baseB + 2 * (G + 1);
        const bool staged = lockstep_stages_sweeps(P_max);
        if (threadIdx.x == 0) s_sweep = atomicAdd(&hdr->sweep_claim, 1);
        __syncthreads();
        for (int32_t c = s_sweep, pos = 0; c < baseB[G];) {
            int32_t next = 0;
            if (threadIdx.x == 0) next = atomicAdd(&hdr->sweep_claim, 1);
            pos = chunk_graph(baseB, G, c, pos);  // claims only grow, so the search moves forward
            const int32_t gi = orderB[pos];
            const int32_t cg = c - baseB[pos];
            sweep_chunk<U>(graphs[gi], items, s, cg, staged, P_max, stage);
            __syncthreads();  // every thread has read s_sweep, and the staged vectors are done with
            if (threadIdx.x == 0) s_sweep = next;
            __syncthreads();
            c = s_sweep;
        }
        // C: recompute of the flagged rows (removal, edge increase)
        const int32_t *baseC = baseB + (G + 1);
        if (baseC[G] > 0) {
            grid_barrier(hdr);
            if (blockIdx.x == 0 && threadIdx.x == 0 && 3 * s + 1 < BATCH_PHASE_STAMPS)
                hdr->phase_ts[3 * s + 1] = wall_clock64();
            // chunks round robin in the sweep phase's graph order (removals
            // largest first, then the edge updates)
            const int32_t *orderC = baseB + 2 * (G + 1);
            for (int32_t c = blockIdx.x, pos = 0; c < baseC[G]; c += gridDim.x) {
                pos = chunk_graph(baseC, G, c, pos);
                const BatchGraph &bg = graphs[orderC[pos]];
                const BatchItem it = items[bg.item_begin + s];
                DevGraph g = bg.g;
                g.n_slots = it.n_slots;
                const int32_t r0 = (c - baseC[pos]) * BATCH_RECOMPUTE_ROWS;
                const int32_t r1 = min(r0 + BATCH_RECOMPUTE_ROWS, it.n_slots);
                // each wavefront uses only its own lists and need bitmap in LDS
                uint32_t *light = lockstep_light_rows(P_max) ? stage + lockstep_light_offset(P_max) : nullptr;
                if (it.op == BOP_REMOVE) {
                    recompute_rows(g, bg, remove_args(bg, it), r0, r1, wlists, nullptr, stage, true, light);
                } else if (it.op == BOP_EDGE && g.ctl->edge_mode == EDGE_INCREASE) {
                    recompute_rows(g, bg, increase_args(g, bg), r0, r1, wlists, nullptr, stage, true, light);
                }
            }
            if (threadIdx.x == 0 && s < BATCH_PHASE_STAMPS)
                atomicMax(reinterpret_cast<unsigned long long *>(&hdr->work_ts[s]), (unsigned long long)wall_clock64());
            grid_barrier(hdr);
            // C2: the deferred heavy rows, one work-group each, taken from a
            // shared counter; a claim maps to (graph, row) through a
            // block-wide scan of the graphs' heavy-row counts, in the same
            // graph order (the largest removals' rows are taken first)
            for (;;) {
                if (threadIdx.x == 0) s_claim = atomicAdd(&hdr->heavy_claim, 1);
                __syncthreads();
                const int32_t t = s_claim;
                int32_t found_g = -1, found_j = 0, base = 0;
                for (int32_t g0 = 0; g0 < G && found_g < 0; g0 += BATCH_THREADS) {
                    const int32_t gi = g0 + threadIdx.x < G ? orderC[g0 + threadIdx.x] : G;
                    int32_t hc = 0;
                    if (gi < G) {
                        const BatchGraph &bq = graphs[gi];
                        const int32_t cnt = bq.item_end - bq.item_begin;
                        if (s < cnt) {
                            const int32_t op = items[bq.item_begin + s].op;
                            if (op == BOP_REMOVE || (op == BOP_EDGE && bq.g.ctl->edge_mode == EDGE_INCREASE))
                                hc = bq.g.ctl->heavy_count;
                        }
                    }
                    int tot;
                    const int off = block_exscan<BATCH_THREADS>(hc, ssh.red, &tot);
                    if (t >= base + off && t < base + off + hc) {
                        s_found_g = gi;
                        s_found_j = t - base - off;
                    }
                    __syncthreads();
                    if (t < base + tot) {
                        found_g = s_found_g;
                        found_j = s_found_j;
                    }
                    base += tot;
                    __syncthreads();
                }
                if (found_g < 0) break;  // block-uniform: every claim beyond the total ends the pass
                const BatchGraph &bg = graphs[found_g];
                const BatchItem it = items[bg.item_begin + s];
                DevGraph g = bg.g;
                g.n_slots = it.n_slots;
                const FusedArgs fa = it.op == BOP_REMOVE ? remove_args(bg, it) : increase_args(g, bg);
                if (lockstep_stages_sweeps(P_max))  // the sweeps' staging area past the need bitmap holds the list
                    heavy_row_block_listed(g, bg, fa, bg.heavy_rows[found_j], stage,
                                           wlists + std::max(4 * 2 * ROW_CAP, (P_max + 31) / 32),
                                           reinterpret_cast<uint32_t *>(wlists), &s_flag, ssh.red);
                else
                    heavy_row_block(g, bg, fa, bg.heavy_rows[found_j], stage, reinterpret_cast<uint32_t *>(wlists),
                                    &s_flag, ssh.red);
            }
        }
        grid_barrier(hdr);
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            atomicExch(&hdr->heavy_claim, 0);
            atomicExch(&hdr->sweep_claim, 0);
        }
        if (blockIdx.x == 0 && threadIdx.x == 0 && 3 * s + 2 < BATCH_PHASE_STAMPS)
            hdr->phase_ts[3 * s + 2] = wall_clock64();
    }
}

// ---------------------------------------------------------------------------
// launches
// ---------------------------------------------------------------------------

size_t batch_lds_bytes(int32_t P_max) { return (2 * (size_t)P_max + 4 * 2 * ROW_CAP) * sizeof(uint32_t); }

// The region after the P_max staging words holds the 4 wave lists of the
// recompute phase, and later the need bitmap of the heavy-row phase (one bit
// per column): whichever is larger.
// A heavy row's list (room for P_max entries) sits past the need bitmap in
// the sweeps' staging area: P_max + max(wave lists, bitmap) + P_max words fit
// in the 2 P_max + 2 LOCKSTEP_STAGE_ROWS words of a staged launch.
static_assert(4 * 2 * ROW_CAP <= 2 * LOCKSTEP_STAGE_ROWS &&
                  (LOCKSTEP_STAGE_MAX_PITCH + 31) / 32 <= 2 * LOCKSTEP_STAGE_ROWS,
              "the heavy-row list fits in the staging area");
size_t batch_lockstep_lds_bytes(int32_t P_max) {
    size_t words = (size_t)P_max + std::max<size_t>(4 * 2 * ROW_CAP, ((size_t)P_max + 31) / 32);
    if (lockstep_stages_sweeps(P_max)) words = std::max<size_t>(words, 2 * (size_t)P_max + 2 * LOCKSTEP_STAGE_ROWS);
    if (lockstep_light_rows(P_max)) words = lockstep_light_offset(P_max) + (BATCH_THREADS / 64) * LIGHT_ROW_WORDS;
    static_assert(LIGHT_ROW_WORDS == LOCKSTEP_LIGHT_WORDS && BATCH_THREADS / 64 == 4, "light-row LDS sizing");
    return words * sizeof(uint32_t);
}

hipError_t configure_batch() {
    static hipError_t status = hipErrorNotReady;
    if (status != hipErrorNotReady) return status;
    const int lds = (int)batch_lds_bytes(BATCH_MAX_CAPACITY);
    // the largest launch: the largest pitch, or the largest one with the
    // light rows' LDS
    int32_t p_light = LOCKSTEP_STAGE_MAX_PITCH;
    while (p_light > 0 && !lockstep_light_rows(p_light)) --p_light;
    const int lds2 = (int)std::max(batch_lockstep_lds_bytes(BATCH_MAX_CAPACITY), batch_lockstep_lds_bytes(p_light));
    status = hipFuncSetAttribute((const void *)k_batch<4>, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    if (status == hipSuccess)
        status = hipFuncSetAttribute((const void *)k_batch<8>, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    if (status == hipSuccess)
        status = hipFuncSetAttribute((const void *)k_batch_lockstep<4>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     lds2);
    if (status == hipSuccess)
        status = hipFuncSetAttribute((const void *)k_batch_lockstep<8>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     lds2);
    if (status == hipSuccess)
        status = hipFuncSetAttribute((const void *)k_batch_lockstep<16>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     lds2);
    (void)hipGetLastError();
    return status;
}

hipError_t launch_batch(BatchHeader *hdr, const BatchGraph *graphs, const int32_t *order, const BatchItem *items,
                        int32_t P_max, int32_t grid, int32_t variant, hipStream_t s) {
    if (P_max > BATCH_MAX_CAPACITY || grid < 1) return hipErrorInvalidValue;
    launch_fill(&hdr->counter, 1, 0, s);
    const size_t lds = batch_lds_bytes(P_max);
    if (variant == 0) k_batch<4><<<grid, BATCH_THREADS, lds, s>>>(hdr, graphs, order, items);
    else k_batch<8><<<grid, BATCH_THREADS, lds, s>>>(hdr, graphs, order, items);
    return hipGetLastError();
}

static const void *lockstep_kernel(int32_t variant) {
    return variant == 2   ? (const void *)k_batch_lockstep<4>
           : variant == 3 ? (const void *)k_batch_lockstep<8>
                          : (const void *)k_batch_lockstep<16>;
}

hipError_t lockstep_grid(int32_t P_max, int32_t variant, int32_t *grid) {
    const size_t lds = batch_lockstep_lds_bytes(P_max);
    int per_cu = 0, dev = 0, cus = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, lockstep_kernel(variant), BATCH_THREADS, lds);
    if (e == hipSuccess) e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    *grid = per_cu * cus;
    return *grid > 0 ? hipSuccess : hipErrorInvalidConfiguration;
}

hipError_t launch_batch_lockstep(BatchHeader *hdr, const BatchGraph *graphs, const BatchItem *items,
                                 const int32_t *tables, int32_t P_max, int32_t grid, int32_t variant, hipStream_t s) {
    if (P_max > BATCH_MAX_CAPACITY || grid < 1) return hipErrorInvalidValue;
    launch_fill(reinterpret_cast<int32_t *>(&hdr->bar_count), 1, 0, s);
    launch_fill(reinterpret_cast<int32_t *>(hdr->bar_group), 8 * 32, 0, s);
    launch_fill(&hdr->err, 1, 0, s);
    launch_fill(&hdr->heavy_claim, 2, 0, s);  // heavy_claim, sweep_claim
    launch_fill(reinterpret_cast<int32_t *>(hdr->work_ts), 2 * BATCH_PHASE_STAMPS, 0, s);
    const size_t lds = batch_lockstep_lds_bytes(P_max);
    void *args[] = {(void *)&hdr, (void *)&graphs, (void *)&items, (void *)&tables};
    const void *fn = lockstep_kernel(variant);
    return hipLaunchCooperativeKernel(fn, dim3(grid), dim3(BATCH_THREADS), args, (unsigned)lds, s);
}

APSP_SR_END
}  // namespace apsp
