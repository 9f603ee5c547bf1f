// Batched updates over many graphs in one persistent launch.
//
// Every work-group pops a graph from a shared counter (largest first by
// default) and applies that graph's queued items in order, so per-graph
// order holds without any wait between work-groups: a work-group exits as
// soon as the counter has passed the last graph.  Each update runs the same
// method as the single-graph kernels, at work-group scope:
//   add node     Corollaries corollary1 / corollary2 (new row / column over
//                the new node's light edges) and Theorem theorem3 (relaxation)
//   remove node  Corollary corollary3 mask, then Bellman-Ford recompute of
//                the flagged entries of each row (one wavefront per row)
//   edge update  decrease: relaxation through the new edge; increase: mask
//                of the pairs that can use the edge, then the same recompute
//   query        Algorithm 7 (candidates, then the canonical walk)
#include <algorithm>

#include "batch_internal.h"
#include "device_common.h"

namespace apsp {

// Visits the 4-column groups of rows [0, n) whose row_ok(i) holds.  Each
// wavefront takes runs of U 256-column chunks (64 lanes x 4 columns, one row
// per chunk), so every lane has U independent 16-byte loads of D in flight
// before it uses any; body(i, c0, ok, d) runs on every lane (ok false where
// the lane has no group), so it may use cross-lane operations.
template <int U, class RowOk, class Body>
__device__ inline void stream_chunks(const DevGraph &g, int32_t n, RowOk row_ok, Body body) {
    const int lane = lane_id(), wv = threadIdx.x >> 6;
    const int32_t Q = (n + 255) >> 8;
    const int32_t total = n * Q;
    for (int32_t base = wv * U; base < total; base += (BATCH_THREADS / 64) * U) {
        uint4 d[U];
        int32_t ri[U], rc[U];
        bool ok[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int32_t k = base + u;
            const int32_t i = k / Q;
            const int32_t c0 = (k - i * Q) * 256 + lane * 4;
            ri[u] = i;
            rc[u] = c0;
            ok[u] = k < total && c0 < n && row_ok(i);
            d[u] = make_uint4(INF, INF, INF, INF);
            if (ok[u]) d[u] = *reinterpret_cast<const uint4 *>(g.D + (int64_t)i * g.ld + c0);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) body(ri[u], rc[u], ok[u], d[u]);
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

// ---------------------------------------------------------------------------
// add node
// ---------------------------------------------------------------------------
constexpr int PREF = 8;  // index entries whose loads are issued together

template <int U>
__device__ void batch_add(const DevGraph &g, const BatchGraph &bg, const BatchItem &it, SelectShared &ssh,
                          uint32_t *stage) {
    const int tid = threadIdx.x;
    const int n = g.n_slots;
    const int32_t p = it.a, new_id = it.b, rank = it.c;
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
        wo[s] = a;
        wi[s] = b;
        if (bad) atomicOr(&g.ctl->err, (int32_t)ERR_VALUE);
    }
    __syncthreads();
    int2 *pin = g.nin + (int64_t)p * NIN_L;
    select_light(wi, n, p, pin, g.nin_cnt + p, g.nin_beta + p, ssh, stage);
    if (!und) select_light(wo, n, p, bg.plist, bg.plist_cnt, bg.plist_beta, ssh, stage);
    const int2 *ol = und ? pin : bg.plist;
    const int ocnt = und ? g.nin_cnt[p] : *bg.plist_cnt;
    const uint32_t obeta = (uint32_t)(und ? g.nin_beta[p] : *bg.plist_beta);
    // new row: out[c] = min_t wo[t] + D[t][c], over p's lightest out-edges first
    {
        const int lim = min(ocnt, g.lim);
        const uint32_t beta_eff = ocnt > g.lim ? (uint32_t)ol[g.lim].y : obeta;
        for (int32_t c = tid; c < n; c += BATCH_THREADS) {
            uint32_t acc = INF;
            if (g.id_of_slot[c] >= 0) {
                // the first PREF entries' loads are issued together; an entry
                // never examined weighs at least the last one examined
                uint32_t pv[PREF];
#pragma unroll
                for (int e = 0; e < PREF; ++e) {
                    const int2 ent = e < lim ? ol[e] : make_int2(0, (int)INF);
                    pv[e] = e < lim ? (uint32_t)ent.y + (uint32_t)g.D[(int64_t)ent.x * g.ld + c] : INF;
                }
#pragma unroll
                for (int e = 0; e < PREF; ++e) acc = min(acc, pv[e]);
                for (int e = PREF; e < lim; ++e) {
                    const int2 ent = ol[e];
                    if ((uint32_t)ent.y >= acc) break;
                    acc = min(acc, (uint32_t)ent.y + (uint32_t)g.D[(int64_t)ent.x * g.ld + c]);
                }
                if (acc > beta_eff)
                    for (int32_t t = 0; t < n; ++t) acc = min(acc, (uint32_t)wo[t] + (uint32_t)g.D[(int64_t)t * g.ld + c]);
            }
            bg.vout[c] = (int32_t)min(acc, INF);
        }
    }
    // new column: in[r] = min_x D[r][x] + wi[x] (directed; = out if undirected)
    if (!und) {
        const int cnt = g.nin_cnt[p];
        const int lim = min(cnt, g.lim);
        const uint32_t beta_eff = cnt > g.lim ? (uint32_t)pin[g.lim].y : (uint32_t)g.nin_beta[p];
        for (int32_t r = tid; r < n; r += BATCH_THREADS) {
            uint32_t best = INF;
            if (g.id_of_slot[r] >= 0) {
                const int32_t *Dr = g.D + (int64_t)r * g.ld;
                uint32_t pv[PREF];
#pragma unroll
                for (int e = 0; e < PREF; ++e) {
                    const int2 ent = e < lim ? pin[e] : make_int2(0, (int)INF);
                    pv[e] = e < lim ? (uint32_t)ent.y + (uint32_t)Dr[ent.x] : INF;
                }
#pragma unroll
                for (int e = 0; e < PREF; ++e) best = min(best, pv[e]);
                for (int e = PREF; e < lim; ++e) {
                    const int2 ent = pin[e];
                    if ((uint32_t)ent.y >= best) break;
                    best = min(best, (uint32_t)ent.y + (uint32_t)Dr[ent.x]);
                }
                if (best > beta_eff)
                    for (int32_t x = 0; x < n; ++x) best = min(best, (uint32_t)Dr[x] + (uint32_t)wi[x]);
            }
            bg.vin[r] = (int32_t)min(best, INF);
        }
    }
    __syncthreads();
    const int32_t *in = und ? bg.vout : bg.vin;
    const int32_t *out = bg.vout;
    // Theorem theorem3 over all old pairs; the new row `out` sits in LDS
    stage_rows(stage, g.P, n, out, nullptr);
    stream_chunks<U>(
        g, n, [&](int32_t i) { return (uint32_t)in[i] < INF; },
        [&](int32_t i, int32_t c0, bool ok, uint4 d) {
            if (!ok) return;
            const uint32_t a = (uint32_t)in[i];
            const uint4 o = *reinterpret_cast<const uint4 *>(stage + c0);
            const uint4 t = make_uint4(a + o.x, a + o.y, a + o.z, a + o.w);
            if (t.x < d.x || t.y < d.y || t.z < d.z || t.w < d.w) {
                d.x = min(d.x, t.x);
                d.y = min(d.y, t.y);
                d.z = min(d.z, t.z);
                d.w = min(d.w, t.w);
                *reinterpret_cast<uint4 *>(g.D + (int64_t)i * g.ld + c0) = d;
            }
        });
    __syncthreads();
    // place row / column p
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
    // p's out-edges are in-edges of every other node
    // (lanes screen 64 lists at a time: an edge at or above a list's bound
    // is not listed)
    for (int32_t y0 = (tid >> 6) * 64; y0 < n; y0 += BATCH_THREADS) {
        const int32_t y = y0 + lane_id();
        const bool cand = y < n && y != p && g.id_of_slot[y] >= 0 && (uint32_t)wo[y] < (uint32_t)g.nin_beta[y];
        unsigned long long m = __ballot(cand);
        while (m) {
            const int b = __ffsll((long long)m) - 1;
            m &= m - 1;
            wave_list_insert(g, y0 + b, p, (uint32_t)wo[y0 + b]);
        }
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------
// mask (removal / increase) and recompute
// ---------------------------------------------------------------------------
// Flags into the graph's bitmap, 32 columns per word per thread step, then
// one wavefront per flagged row runs the Bellman-Ford recompute in place.
template <int U>
__device__ void batch_mask_recompute(const DevGraph &g, const BatchGraph &bg, const FusedArgs &fa, uint32_t w_old,
                                     uint32_t *stage, int32_t *wlists) {
    const int tid = threadIdx.x, lane = lane_id(), wv = tid >> 6;
    const int n = g.n_slots;
    const int nw = (n + 31) / 32;
    const int64_t nwp = (g.P + 31) / 32;
    // the pair test's row vectors in LDS; rows stream through in chunks and
    // 8 lanes assemble each 32-column flag word with shuffles
    stage_rows(stage, g.P, n, fa.row1, fa.row2);
    const uint32_t *S1 = stage, *S2 = stage + g.P;
    stream_chunks<U>(
        g, n,
        [&](int32_t i) {
            const RowTests rt = row_tests(g, fa, i, w_old);
            return rt.t1 || rt.t2;
        },
        [&](int32_t i, int32_t c0, bool ok, uint4 d) {
            uint32_t bits = 0;
            if (ok) {
                const RowTests rt = row_tests(g, fa, i, w_old);
                const uint4 v1 = *reinterpret_cast<const uint4 *>(S1 + c0);
                const uint4 v2 = fa.row2 ? *reinterpret_cast<const uint4 *>(S2 + c0) : v1;
                const uint32_t dv[4] = {d.x, d.y, d.z, d.w};
                const uint32_t w1[4] = {v1.x, v1.y, v1.z, v1.w};
                const uint32_t w2[4] = {v2.x, v2.y, v2.z, v2.w};
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int32_t j = c0 + e;
                    const bool f = j < n && j != i && !(fa.mode == FUSED_REMOVE && j == fa.k) && dv[e] < INF &&
                                   ((rt.t1 && rt.a1 + w1[e] == dv[e]) || (rt.t2 && rt.a2 + w2[e] == dv[e]));
                    bits |= (uint32_t)f << e;
                }
            }
            uint32_t word = bits << ((lane & 7) * 4);
#pragma unroll
            for (int o = 1; o < 8; o <<= 1) word |= (uint32_t)__shfl_xor((int)word, o);
            if (ok && (lane & 7) == 0) bg.flag_bits[(int64_t)i * nwp + (c0 >> 5)] = word;
            if (__ballot(ok && word != 0) != 0 && lane == 0) atomicOr(&bg.row_bits[i >> 5], 1u << (i & 31));
        });
    __syncthreads();
    int my_flagged = 0, my_rows = 0, my_fs = 0, my_sweeps = 0;
    int32_t *list = wlists + wv * 2 * ROW_CAP;
    int32_t *fsl = list + ROW_CAP;
    int32_t *glist = bg.scratch + (int64_t)wv * 2 * g.P;  // rows with more than ROW_CAP flags
    int32_t *gfsl = glist + g.P;
    for (int32_t i0 = wv * 64; i0 < n; i0 += BATCH_THREADS) {
      const int32_t ii = i0 + lane;
      unsigned long long rows = __ballot(ii < n && ((bg.row_bits[ii >> 5] >> (ii & 31)) & 1u));
      while (rows) {
        const int32_t i = i0 + __ffsll((long long)rows) - 1;
        rows &= rows - 1;
        const uint32_t *fw = bg.flag_bits + (int64_t)i * nwp;
        int cnt = 0;
        for (int b = 0; b < nw; b += 64) {
            const int w = b + lane;
            const uint32_t bits0 = w < nw ? fw[w] : 0u;
            const int c = __popc(bits0);
            int incl = c;
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
                const int t = __shfl_up(incl, o);
                if (lane >= o) incl += t;
            }
            cnt += __shfl(incl, 63);
        }
        int32_t *L = cnt <= ROW_CAP ? list : glist;
        int32_t *F = cnt <= ROW_CAP ? fsl : gfsl;
        int done = 0;
        for (int b = 0; b < nw; b += 64) {
            const int w = b + lane;
            uint32_t bits = w < nw ? fw[w] : 0u;
            const int c = __popc(bits);
            int incl = c;
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
                const int t = __shfl_up(incl, o);
                if (lane >= o) incl += t;
            }
            int pos = done + incl - c;
            while (bits) {
                const int bt = __ffs(bits) - 1;
                bits &= bits - 1;
                L[pos++] = w * 32 + bt;
            }
            done += __shfl(incl, 63);
        }
        __threadfence_block();
        int32_t *Drow = g.D + (int64_t)i * g.ld;
        for (int e = lane; e < cnt; e += 64) Drow[L[e]] = (int32_t)INF;
        if (fa.mode == FUSED_REMOVE && lane == 0) Drow[fa.k] = (int32_t)INF;
        __threadfence_block();
        int sweeps = 0;
        wave_bellman_ford(g, Drow, L, cnt, F, sweeps, my_fs);
        my_sweeps = max(my_sweeps, sweeps);
        my_flagged += cnt;
        ++my_rows;
      }
    }
    __syncthreads();
    for (int w = tid; w < (n + 31) / 32; w += BATCH_THREADS) bg.row_bits[w] = 0;
    if (lane == 0 && (my_rows || my_fs)) {
        atomicAdd(&g.ctl->flagged, (unsigned long long)my_flagged);
        atomicAdd(&g.ctl->rows, my_rows);
        atomicAdd(&g.ctl->full_scans, my_fs);
        atomicMax(&g.ctl->sweeps, my_sweeps);
    }
    __syncthreads();
}

// Rebuild the index lists of y when they have shrunk (block-wide select).
__device__ void batch_rebuild_if_short(const DevGraph &g, int32_t y, SelectShared &ssh, uint32_t *stage) {
    if (!(g.nin_cnt[y] < NIN_L / 2 && (uint32_t)g.nin_beta[y] < INF && g.id_of_slot[y] >= 0)) return;
    select_light(in_matrix(g) + (int64_t)y * g.ld, g.n_slots, y, g.nin + (int64_t)y * NIN_L, g.nin_cnt + y,
                 g.nin_beta + y, ssh, stage);
}

template <int U>
__device__ void batch_remove(const DevGraph &g, const BatchGraph &bg, const BatchItem &it, SelectShared &ssh,
                             uint32_t *stage, int32_t *wlists) {
    const int tid = threadIdx.x;
    const int n = g.n_slots;
    const int32_t k = it.a, rank = it.b, n_live = it.c;
    for (int32_t i = tid; i < n; i += BATCH_THREADS) {
        bg.colu[i] = g.D[(int64_t)i * g.ld + k];
        bg.rowu[i] = g.D[(int64_t)k * g.ld + i];
    }
    __syncthreads();
    FusedArgs fa{};
    fa.mode = FUSED_REMOVE;
    fa.k = k;
    fa.col1 = bg.colu;
    fa.row1 = bg.rowu;
    fa.row2 = nullptr;
    batch_mask_recompute<U>(g, bg, fa, 0, stage, wlists);
    // drop k from every index list (lanes screen 64 lists at a time: k can
    // be listed in y only if its edge is no heavier than y's last entry);
    // k's own list empties
    for (int32_t y0 = (tid >> 6) * 64; y0 < n; y0 += BATCH_THREADS) {
        const int32_t y = y0 + lane_id();
        bool cand = false;
        if (y < n && y != k) {
            const int c = g.nin_cnt[y];
            const uint32_t wk = (uint32_t)g.A[(int64_t)k * g.ld + y];
            cand = c > 0 && wk < INF && wk <= (uint32_t)g.nin[(int64_t)y * NIN_L + c - 1].y;
        }
        unsigned long long m = __ballot(cand);
        while (m) {
            const int b = __ffsll((long long)m) - 1;
            m &= m - 1;
            wave_list_purge(g, y0 + b, k);
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
    // tombstone
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
    // ranks after the removed one move down by one
    for (int32_t t = tid; t < n_live - 1; t += BATCH_THREADS) it.rank_dst[t] = it.rank_src[t < rank ? t : t + 1];
    __syncthreads();
}

template <int U>
__device__ void batch_edge(const DevGraph &g, const BatchGraph &bg, const BatchItem &it, SelectShared &ssh,
                           uint32_t *stage, int32_t *wlists) {
    const int tid = threadIdx.x;
    const int n = g.n_slots;
    const int32_t su = it.a, sv = it.b, w = it.c;
    if (tid < 64) edge_begin_wave(g, su, sv, w);
    __syncthreads();
    const int32_t mode = g.ctl->edge_mode;
    const uint32_t w_old = (uint32_t)g.ctl->w_old;
    if (mode != EDGE_NOOP) {
        for (int32_t i = tid; i < n; i += BATCH_THREADS) {
            bg.colu[i] = g.D[(int64_t)i * g.ld + su];
            bg.colv[i] = g.D[(int64_t)i * g.ld + sv];
            bg.rowu[i] = g.D[(int64_t)su * g.ld + i];
            bg.rowv[i] = g.D[(int64_t)sv * g.ld + i];
        }
        __syncthreads();
    }
    if (mode == EDGE_DECREASE) {
        // relaxation through the new edge: D[i][j] vs D[i][u] + w + D[v][j]
        // (and D[i][v] + w + D[u][j] when undirected), rows filtered first
        const bool und = g.undirected != 0;
        const uint32_t wn = (uint32_t)w;
        stage_rows(stage, g.P, n, bg.rowv, und ? bg.rowu : nullptr);
        const uint32_t *SV = stage, *SU = stage + g.P;
        stream_chunks<U>(
            g, n,
            [&](int32_t i) {
                const uint32_t du = (uint32_t)bg.colu[i], dv = (uint32_t)bg.colv[i];
                return du + wn < dv || (und && dv + wn < du);
            },
            [&](int32_t i, int32_t c0, bool ok, uint4 d) {
                if (!ok) return;
                const uint32_t du = (uint32_t)bg.colu[i], dv = (uint32_t)bg.colv[i];
                const uint32_t x1 = du + wn < dv ? du + wn : INF;
                const uint32_t x2 = und && dv + wn < du ? dv + wn : INF;
                const uint4 rv = *reinterpret_cast<const uint4 *>(SV + c0);
                uint4 ru = make_uint4(INF, INF, INF, INF);
                if (und) ru = *reinterpret_cast<const uint4 *>(SU + c0);
                const uint4 t = make_uint4(min(x1 + rv.x, x2 + ru.x), min(x1 + rv.y, x2 + ru.y),
                                           min(x1 + rv.z, x2 + ru.z), min(x1 + rv.w, x2 + ru.w));
                if (t.x < d.x || t.y < d.y || t.z < d.z || t.w < d.w) {
                    d.x = min(d.x, t.x);
                    d.y = min(d.y, t.y);
                    d.z = min(d.z, t.z);
                    d.w = min(d.w, t.w);
                    *reinterpret_cast<uint4 *>(g.D + (int64_t)i * g.ld + c0) = d;
                }
            });
        __syncthreads();
    } else if (mode == EDGE_INCREASE) {
        FusedArgs fa{};
        fa.mode = FUSED_INCREASE;
        fa.k = -1;
        fa.col1 = bg.colu;
        fa.col2 = bg.colv;
        fa.row1 = bg.rowv;
        fa.row2 = g.undirected ? bg.rowu : nullptr;
        batch_mask_recompute<U>(g, bg, fa, w_old, stage, wlists);
    }
    batch_rebuild_if_short(g, sv, ssh, stage);
    if (g.undirected) batch_rebuild_if_short(g, su, ssh, stage);
    __syncthreads();
}

// ---------------------------------------------------------------------------
// the persistent kernel
// ---------------------------------------------------------------------------
template <int U>
__global__ __launch_bounds__(BATCH_THREADS, 2) void k_batch(BatchHeader *hdr, const BatchGraph *graphs,
                                                         const int32_t *order, const BatchItem *items) {
    extern __shared__ uint32_t stage[];  // 2 P words of row vectors / select staging, then 4 wave lists of 2 ROW_CAP
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
            if (threadIdx.x == 0) {
                g.ctl->flagged = 0;
                g.ctl->rows = 0;
                g.ctl->full_scans = 0;
                g.ctl->sweeps = 0;
            }
            __syncthreads();
            switch (it.op) {
            case BOP_ADD: batch_add<U>(g, bg, it, ssh, stage); break;
            case BOP_REMOVE: batch_remove<U>(g, bg, it, ssh, stage, wlists); break;
            case BOP_EDGE: batch_edge<U>(g, bg, it, ssh, stage, wlists); break;
            case BOP_QUERY: query_block(g, it.a, it.b, it.out, bg.qscratch); break;
            default: break;
            }
            __syncthreads();
        }
        if (threadIdx.x == 0) hdr->times[2 * bg.index + 1] = wall_clock64();
    }
}

size_t batch_lds_bytes(int32_t P_max) { return (2 * (size_t)P_max + 4 * 2 * ROW_CAP) * sizeof(uint32_t); }

hipError_t configure_batch() {
    static hipError_t status = hipErrorNotReady;
    if (status != hipErrorNotReady) return status;
    const int lds = (int)batch_lds_bytes(BATCH_MAX_CAPACITY);
    status = hipFuncSetAttribute((const void *)k_batch<4>, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    if (status == hipSuccess)
        status = hipFuncSetAttribute((const void *)k_batch<8>, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
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

}  // namespace apsp
