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

// ---------------------------------------------------------------------------
// add node
// ---------------------------------------------------------------------------
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
                for (int e = 0; e < lim; ++e) {
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
                for (int e = 0; e < lim; ++e) {
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
    // Theorem theorem3 over all old pairs, (row, 4-column) cells spread over the block
    const int nc4 = (n + 3) / 4;
    const int64_t cells = (int64_t)n * nc4;
#pragma unroll U
    for (int64_t x = tid; x < cells; x += BATCH_THREADS) {
        const int32_t i = (int32_t)(x / nc4);
        const int32_t c0 = (int32_t)(x - (int64_t)i * nc4) * 4;
        const uint32_t a = (uint32_t)in[i];
        if (a >= INF) continue;
        uint4 *dp = reinterpret_cast<uint4 *>(g.D + (int64_t)i * g.ld + c0);
        uint4 d = *dp;
        const uint32_t o[4] = {(uint32_t)out[c0], c0 + 1 < n ? (uint32_t)out[c0 + 1] : INF,
                               c0 + 2 < n ? (uint32_t)out[c0 + 2] : INF, c0 + 3 < n ? (uint32_t)out[c0 + 3] : INF};
        const uint4 t = make_uint4(a + o[0], a + o[1], a + o[2], a + o[3]);
        if (t.x < d.x || t.y < d.y || t.z < d.z || t.w < d.w) {
            d.x = min(d.x, t.x);
            d.y = min(d.y, t.y);
            d.z = min(d.z, t.z);
            d.w = min(d.w, t.w);
            *dp = d;
        }
    }
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
    for (int32_t y = tid >> 6; y < n; y += BATCH_THREADS / 64)
        if (y != p && g.id_of_slot[y] >= 0) wave_list_insert(g, y, p, (uint32_t)wo[y]);
    __syncthreads();
}

// ---------------------------------------------------------------------------
// mask (removal / increase) and recompute
// ---------------------------------------------------------------------------
// Flags into the graph's bitmap, 32 columns per word per thread step, then
// one wavefront per flagged row runs the Bellman-Ford recompute in place.
template <int U>
__device__ void batch_mask_recompute(const DevGraph &g, const BatchGraph &bg, const FusedArgs &fa, uint32_t w_old,
                                     int32_t *wlists) {
    const int tid = threadIdx.x, lane = lane_id(), wv = tid >> 6;
    const int n = g.n_slots;
    const int nw = (n + 31) / 32;
    const int64_t nwp = (g.P + 31) / 32;
    const int64_t cells = (int64_t)n * nw;
#pragma unroll U
    for (int64_t x = tid; x < cells; x += BATCH_THREADS) {
        const int32_t i = (int32_t)(x / nw);
        const int32_t w = (int32_t)(x - (int64_t)i * nw);
        const RowTests rt = row_tests(g, fa, i, w_old);
        if (!rt.t1 && !rt.t2) continue;
        const uint32_t a1 = rt.t1 ? rt.a1 : 0x80000000u, a2 = rt.t2 ? rt.a2 : 0x80000000u;
        const int32_t *Dr = g.D + (int64_t)i * g.ld + w * 32;
        const int32_t *R1 = fa.row1 + w * 32;
        const int32_t *R2 = fa.row2 ? fa.row2 + w * 32 : R1;
        uint32_t word = 0;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const uint4 d = *reinterpret_cast<const uint4 *>(Dr + 4 * q);
            const uint4 v1 = *reinterpret_cast<const uint4 *>(R1 + 4 * q);
            const uint4 v2 = *reinterpret_cast<const uint4 *>(R2 + 4 * q);
            const uint32_t dv[4] = {d.x, d.y, d.z, d.w};
            const uint32_t w1[4] = {v1.x, v1.y, v1.z, v1.w};
            const uint32_t w2[4] = {v2.x, v2.y, v2.z, v2.w};
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const bool f = dv[e] < INF && (a1 + w1[e] == dv[e] || a2 + w2[e] == dv[e]);
                word |= (uint32_t)f << (4 * q + e);
            }
        }
        const int32_t j0 = w * 32;
        if ((unsigned)(i - j0) < 32u) word &= ~(1u << (i - j0));
        if (fa.mode == FUSED_REMOVE && (unsigned)(fa.k - j0) < 32u) word &= ~(1u << (fa.k - j0));
        if (j0 + 32 > n) word &= (n - j0 >= 32) ? ~0u : ((1u << (n - j0)) - 1u);
        bg.flag_bits[(int64_t)i * nwp + w] = word;
        if (word) atomicOr(&bg.row_bits[i >> 5], 1u << (i & 31));
    }
    __syncthreads();
    int my_flagged = 0, my_rows = 0, my_fs = 0, my_sweeps = 0;
    int32_t *list = wlists + wv * 2 * ROW_CAP;
    int32_t *fsl = list + ROW_CAP;
    int32_t *glist = bg.scratch + (int64_t)wv * 2 * g.P;  // rows with more than ROW_CAP flags
    int32_t *gfsl = glist + g.P;
    for (int32_t i = wv; i < n; i += BATCH_THREADS / 64) {
        if (((bg.row_bits[i >> 5] >> (i & 31)) & 1u) == 0) continue;
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
    batch_mask_recompute<U>(g, bg, fa, 0, wlists);
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
    __syncthreads();
    if (tid == 0) g.id_of_slot[k] = -1;
    // drop k from every index list; k's own list empties
    for (int32_t y = tid >> 6; y < n; y += BATCH_THREADS / 64) {
        if (y == k) {
            g.nin[(int64_t)y * NIN_L + lane_id()] = make_int2(0, (int)INF);
            if (lane_id() == 0) { g.nin_cnt[y] = 0; g.nin_beta[y] = (int32_t)INF; }
        } else {
            wave_list_purge(g, y, k);
        }
    }
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
        const bool und = g.undirected != 0;
        const uint32_t wn = (uint32_t)w;
        const int nc4 = (n + 3) / 4;
        const int64_t cells = (int64_t)n * nc4;
#pragma unroll U
        for (int64_t x = tid; x < cells; x += BATCH_THREADS) {
            const int32_t i = (int32_t)(x / nc4);
            const int32_t c0 = (int32_t)(x - (int64_t)i * nc4) * 4;
            const uint32_t du = (uint32_t)bg.colu[i], dv = (uint32_t)bg.colv[i];
            const uint32_t a1 = du + wn, a2 = dv + wn;
            const bool t1 = a1 < dv, t2 = und && a2 < du;
            if (!t1 && !t2) continue;
            const uint32_t x1 = t1 ? a1 : INF, x2 = t2 ? a2 : INF;
            int32_t *Dr = g.D + (int64_t)i * g.ld;
            for (int e = 0; e < 4 && c0 + e < n; ++e) {
                const int32_t j = c0 + e;
                const uint32_t t = min(x1 + (uint32_t)bg.rowv[j], und ? x2 + (uint32_t)bg.rowu[j] : INF);
                if (t < (uint32_t)Dr[j]) Dr[j] = (int32_t)t;
            }
        }
        __syncthreads();
    } else if (mode == EDGE_INCREASE) {
        FusedArgs fa{};
        fa.mode = FUSED_INCREASE;
        fa.k = -1;
        fa.col1 = bg.colu;
        fa.col2 = bg.colv;
        fa.row1 = bg.rowv;
        fa.row2 = g.undirected ? bg.rowu : nullptr;
        batch_mask_recompute<U>(g, bg, fa, w_old, wlists);
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
    extern __shared__ uint32_t stage[];  // select staging (P words), then 4 wave lists of 2 ROW_CAP
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
        int32_t *wlists = reinterpret_cast<int32_t *>(stage) + bg.g.P;
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

size_t batch_lds_bytes(int32_t P_max) { return ((size_t)P_max + 4 * 2 * ROW_CAP) * sizeof(uint32_t); }

hipError_t configure_batch() {
    static hipError_t status = hipErrorNotReady;
    if (status != hipErrorNotReady) return status;
    const int lds = (int)batch_lds_bytes(BATCH_MAX_CAPACITY);
    status = hipFuncSetAttribute((const void *)k_batch<1>, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    if (status == hipSuccess)
        status = hipFuncSetAttribute((const void *)k_batch<2>, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    (void)hipGetLastError();
    return status;
}

hipError_t launch_batch(BatchHeader *hdr, const BatchGraph *graphs, const int32_t *order, const BatchItem *items,
                        int32_t P_max, int32_t grid, int32_t variant, hipStream_t s) {
    if (P_max > BATCH_MAX_CAPACITY || grid < 1) return hipErrorInvalidValue;
    launch_fill(&hdr->counter, 1, 0, s);
    const size_t lds = batch_lds_bytes(P_max);
    if (variant == 0) k_batch<1><<<grid, BATCH_THREADS, lds, s>>>(hdr, graphs, order, items);
    else k_batch<2><<<grid, BATCH_THREADS, lds, s>>>(hdr, graphs, order, items);
    return hipGetLastError();
}

}  // namespace apsp
