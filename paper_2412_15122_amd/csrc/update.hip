// Warm-start updates: add node, remove node, edge decrease / increase, and the
// light in-edge index they share.
//
// Notation: a (+) b = cat(a, b), the concatenation of the semiring the unit
// is compiled for (a + b for shortest paths, max(a, b) for minimax paths),
// INF = 2^30, evaluated in uint32 (no wrap, and a min against a value <= INF
// needs no clamp).
#include <algorithm>

#include "device_common.h"

namespace apsp {
APSP_SR_BEGIN

// Zero the per-update counters (the edge decision is written by k_edge_begin).
__device__ __forceinline__ void reset_stats(Ctl *c) {
    c->flagged = 0;
    c->rows = 0;
    c->full_scans = 0;
    c->sweeps = 0;
    c->rows_relaxed = 0;
    c->scope_r = 0;
    c->scope_c = 0;
    c->short_count = 0;
    c->heavy_count = 0;
    c->changed = 0;
    c->rows_changed = 0;
}

// ---------------------------------------------------------------------------
// light in-edge index
// ---------------------------------------------------------------------------
// For node y the index lists up to NIN_L in-edges (x, w) with the smallest
// weights, ascending, and a bound beta[y] <= the weight of every unlisted
// in-edge (INF when every in-edge is listed).  Scans that stop at
// min(cnt, lim) entries use beta_eff = (cnt > lim) ? list[lim].w : beta.

// Build the index of nodes first .. first+count-1 from row y of the in-edge
// matrix.  only_short: rebuild only lists that have shrunk below NIN_L/2
// while unlisted in-edges exist.
__device__ __forceinline__ void nin_build_one(const DevGraph &g, int32_t y, int32_t only_short, SelectShared &sh,
                                              uint32_t *stage) {
    if (y < 0 || y >= g.n_slots) return;
    int32_t *cnt = g.nin_cnt + y, *beta = g.nin_beta + y;
    if (only_short && !(*cnt < NIN_L / 2 && (uint32_t)*beta < INF)) return;
    int2 *list = g.nin + (int64_t)y * NIN_L;
    if (g.A[(int64_t)y * g.ld + y] != 0) {  // dead slot
        if (threadIdx.x == 0) { *cnt = 0; *beta = (int32_t)INF; }
        return;
    }
    select_light(in_matrix(g) + (int64_t)y * g.ld, g.n_slots, y, list, cnt, beta, sh, stage);
}

__global__ __launch_bounds__(256) void k_nin_build(DevGraph g, int32_t first, int32_t only_short) {
    __shared__ SelectShared sh;
    extern __shared__ uint32_t stage[];
    nin_build_one(g, first + blockIdx.x, only_short, sh, stage);
}

template <int NT>
__device__ __forceinline__ void mask_finish_block(const DevGraph &g, const int32_t *partials, int32_t blocks,
                                                  uint32_t *red);

// The statistics of an edge update's recompute: a tight increase's partials
// of `blocks` work-groups summed into the control block (nothing for other
// edge updates).  One work-group, launched only when the statistics are read.
__global__ __launch_bounds__(256) void k_edge_stats(DevGraph g, const int32_t *partials, int32_t blocks) {
    __shared__ uint32_t red[8];
    if (blocks != 0 && g.ctl->edge_mode == EDGE_INCREASE) mask_finish_block<256>(g, partials, blocks, red);
}

size_t nin_build_lds_bytes(int32_t P) { return (size_t)P * sizeof(uint32_t); }

void launch_nin_build(const DevGraph &g, int32_t first, int32_t count, int32_t only_short, hipStream_t s) {
    if (count <= 0) return;
    k_nin_build<<<count, 256, nin_build_lds_bytes(g.P), s>>>(g, first, only_short);
}

void launch_edge_stats(const DevGraph &g, const int32_t *partials, int32_t blocks, hipStream_t s) {
    k_edge_stats<<<1, 256, 0, s>>>(g, partials, blocks);
}

// A single list on the critical path of an update: one wide block, so that
// more loads are in flight and the LDS passes take fewer steps.
constexpr int SELECT_WIDE = 1024;

__global__ __launch_bounds__(SELECT_WIDE) void k_select_vec(const int32_t *vals, int32_t n, int32_t excl, int2 *list,
                                                            int32_t *cnt, int32_t *beta) {
    __shared__ SelectShared sh;
    extern __shared__ uint32_t stage[];
    select_light<SELECT_WIDE>(vals, n, excl, list, cnt, beta, sh, stage);
}

void launch_select_vec(const int32_t *vals, int32_t n, int32_t exclude, int2 *list, int32_t *cnt,
                       int32_t *beta, hipStream_t s) {
    k_select_vec<<<1, SELECT_WIDE, (size_t)(n > 0 ? n : 1) * sizeof(uint32_t), s>>>(vals, n, exclude, list, cnt,
                                                                                    beta);
}



__global__ __launch_bounds__(SELECT_WIDE) void k_nin_rebuild_queue(DevGraph g, const int32_t *queue) {
    __shared__ SelectShared sh;
    extern __shared__ uint32_t stage[];
    const int count = g.ctl->short_count;
    for (int idx = blockIdx.x; idx < count; idx += gridDim.x) {
        const int32_t y = queue[idx];
        select_light<SELECT_WIDE>(in_matrix(g) + (int64_t)y * g.ld, g.n_slots, y, g.nin + (int64_t)y * NIN_L,
                                  g.nin_cnt + y, g.nin_beta + y, sh, stage);
    }
}

void launch_nin_rebuild_queue(const DevGraph &g, const int32_t *queue, hipStream_t s) {
    if (g.n_slots <= 0) return;
    k_nin_rebuild_queue<<<32, SELECT_WIDE, nin_build_lds_bytes(g.P), s>>>(g, queue);
}

// ---------------------------------------------------------------------------
// add node (Section 3.1)
// ---------------------------------------------------------------------------

// wo[s] / wi[s]: the new node's out- / in-weight towards slot s (INF for
// dead slots); weights outside [0, INF] become INF and set the sticky error.
__global__ void k_scatter_weights(DevGraph g, const int32_t *__restrict__ w_out, const int32_t *__restrict__ w_in,
                                  const int32_t *__restrict__ slot_of_rank, int32_t n_live, int32_t *wo,
                                  int32_t *wi) {
    int32_t r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r == 0) reset_stats(g.ctl);  // the start of an addition
    // dead slots (the new slot among them) have no edges; live slots are
    // written below by the thread of their rank, so no slot is written twice
    if (r < g.n_slots && g.id_of_slot[r] < 0) {
        wo[r] = (int32_t)INF;
        wi[r] = (int32_t)INF;
    }
    if (r >= n_live) return;
    int32_t s = slot_of_rank[r];
    int32_t a = w_out[r];
    int32_t b = w_in ? w_in[r] : a;
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

void launch_scatter_weights(const DevGraph &g, const int32_t *w_out, const int32_t *w_in,
                            const int32_t *slot_of_rank, int32_t n_live, int32_t *wo, int32_t *wi,
                            hipStream_t s) {
    const int32_t threads = std::max(g.n_slots, n_live);
    k_scatter_weights<<<(threads + 255) / 256, 256, 0, s>>>(g, w_out, g.undirected ? nullptr : w_in, slot_of_rank,
                                                           n_live, wo, wi);
}

// out[c] = min_t wo[t] (+) D[t][c]  (Corollary 1: SPD(p, c)).
// The new node's lightest out-edges (plist, ascending weight) are split over
// the block's 16 waves, each reading its (at most four) rows' chunks at once
// -- one round trip, at most 64 rows of 1 KB per block.  Every unlisted t
// has wo[t] >= beta, so a column whose value is <= beta is final; columns
// above beta (or unreachable) take an exhaustive scan.  One block = 256
// columns, a lane 4 of them.
constexpr int ADD_OUT_THREADS = 1024;
constexpr int ADD_OUT_WAVES = ADD_OUT_THREADS / 64;
static_assert(ADD_OUT_WAVES * 4 >= NIN_L, "four list entries per wave cover the list");
__global__ __launch_bounds__(ADD_OUT_THREADS) void k_add_out(DevGraph g, const int2 *__restrict__ plist,
                                                             const int32_t *__restrict__ pcnt,
                                                             const int32_t *__restrict__ pbeta,
                                                             const int32_t *__restrict__ wo, int32_t *__restrict__ out) {
    __shared__ uint32_t part[ADD_OUT_WAVES][256];
    __shared__ uint32_t red[ADD_OUT_WAVES];
    const int n = g.n_slots;
    const int tid = threadIdx.x, lane = lane_id(), wv = tid >> 6;
    const int32_t cbase = blockIdx.x * 256;
    const int32_t c0 = cbase + lane * 4;
    const int cnt = *pcnt;
    const int lim = min(cnt, g.lim);
    const uint32_t beta_eff = cnt > g.lim ? (uint32_t)plist[g.lim].y : (uint32_t)*pbeta;
    uint32_t acc[4] = {INF, INF, INF, INF};
    if (c0 < n) {
        int2 ent[4];
        int4 v[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int e = wv + q * ADD_OUT_WAVES;
            ent[q] = e < lim ? plist[e] : make_int2(0, (int)INF);
        }
#pragma unroll
        for (int q = 0; q < 4; ++q)
            if ((uint32_t)ent[q].y < INF) v[q] = *reinterpret_cast<const int4 *>(g.D + (int64_t)ent[q].x * g.ld + c0);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            if ((uint32_t)ent[q].y >= INF) continue;
            const uint32_t w = (uint32_t)ent[q].y;
            acc[0] = min(acc[0], cat(w, (uint32_t)v[q].x));
            acc[1] = min(acc[1], cat(w, (uint32_t)v[q].y));
            acc[2] = min(acc[2], cat(w, (uint32_t)v[q].z));
            acc[3] = min(acc[3], cat(w, (uint32_t)v[q].w));
        }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) part[wv][lane * 4 + q] = acc[q];
    __syncthreads();
    const int32_t c = cbase + tid;  // one column per thread of the first 256 from here on
    uint32_t fin = INF;
    if (tid < 256) {
#pragma unroll
        for (int w = 0; w < ADD_OUT_WAVES; ++w) fin = min(fin, part[w][tid]);
    }
    const bool live_c = tid < 256 && c < n && g.id_of_slot[c] >= 0;
    const int need = block_sum<ADD_OUT_THREADS>(live_c && fin > beta_eff, red);
    if (need && tid < 256 && c < n)
        for (int32_t t = 0; t < n; ++t) fin = min(fin, cat((uint32_t)wo[t], (uint32_t)g.D[(int64_t)t * g.ld + c]));
    if (tid < 256 && c < n) out[c] = (int32_t)min(fin, INF);
}

void launch_add_out(const DevGraph &g, const int2 *plist, const int32_t *pcnt, const int32_t *pbeta,
                    const int32_t *wo, int32_t *out, hipStream_t s) {
    if (g.n_slots <= 0) return;
    k_add_out<<<(g.n_slots + 255) / 256, ADD_OUT_THREADS, 0, s>>>(g, plist, pcnt, pbeta, wo, out);
}

// in[i] = min_r D[i][r] (+) wi[r]  (Corollary 2: SPD(i, p)), one wave
// per row over the new node's light in-edges (its own index list, built
// from wi), exhaustive when the row's value exceeds beta.  Directed only;
// for an undirected graph in = out.
__global__ __launch_bounds__(256) void k_add_in(DevGraph g, int32_t p, const int32_t *__restrict__ wi,
                                                int32_t *__restrict__ in) {
    const int32_t i = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = lane_id();
    if (i >= g.n_slots) return;
    if (g.id_of_slot[i] < 0) {
        if (lane == 0) in[i] = (int32_t)INF;
        return;
    }
    const int2 *L = g.nin + (int64_t)p * NIN_L;
    const int cnt = g.nin_cnt[p];
    const int lim = min(cnt, g.lim);
    const uint32_t beta_eff = cnt > g.lim ? (uint32_t)L[g.lim].y : (uint32_t)g.nin_beta[p];
    const int32_t *Di = g.D + (int64_t)i * g.ld;
    uint32_t best = INF;
    if (lane < lim) {
        int2 ent = L[lane];
        best = cat((uint32_t)ent.y, (uint32_t)Di[ent.x]);
    }
    best = wave_min(best);
    if (best > beta_eff) best = wave_min_plus_below(Di, wi, g.n_slots, best);  // only weights below best matter
    if (lane == 0) in[i] = (int32_t)min(best, INF);
}

void launch_add_in(const DevGraph &g, int32_t p, const int32_t *wi, int32_t *in, hipStream_t s) {
    if (g.n_slots <= 0) return;
    k_add_in<<<(g.n_slots + 3) / 4, 256, 0, s>>>(g, p, wi, in);
}

// Row-stationary streaming, for the edge update's sweep and the count-only
// removal mask: a work-group owns SWEEP_ROWS consecutive rows, evaluates
// their row-side values once, then walks the rows' columns in tiles of 1024
// (256 lanes x 4 columns), loading each tile's rows of D (non-temporal: D is
// streamed once) together with the slices of the row vectors, so a tile
// waits on one round trip.  (The add relaxation and the removal mask, which
// sweep every row, keep one tile per work-group: over the whole matrix
// that order streams D faster on this part.)  The tile count is the same for
// every lane of a wavefront (lanes past n load nothing), so the cross-lane
// steps of a tile body see every lane.
constexpr int SWEEP_ROWS = 8;

template <int R>
struct SweepTile {
    uint4 d[R];
    uint4 v1, v2;
};

// 4 consecutive entries of a row vector at c0 (INF from column n on).
__device__ __forceinline__ uint4 vec_slice(const int32_t *v, int32_t c0, int32_t n) {
    if (c0 + 3 < n) return *reinterpret_cast<const uint4 *>(v + c0);
    return make_uint4(c0 < n ? (uint32_t)v[c0] : INF, c0 + 1 < n ? (uint32_t)v[c0 + 1] : INF,
                      c0 + 2 < n ? (uint32_t)v[c0 + 2] : INF, c0 + 3 < n ? (uint32_t)v[c0 + 3] : INF);
}

// Loads of one tile: rows r0 + r with bit r of `act`, and the slices of v1
// (and v2 when given) at column c0.
template <int R>
__device__ __forceinline__ void sweep_load(SweepTile<R> &t, const DevGraph &g, int32_t r0, uint32_t act, int32_t c0,
                                           int32_t n, const int32_t *v1, const int32_t *v2) {
    const bool ok = c0 < n;
    t.v1 = ok ? vec_slice(v1, c0, n) : make_uint4(INF, INF, INF, INF);
    t.v2 = ok && v2 ? vec_slice(v2, c0, n) : make_uint4(INF, INF, INF, INF);
#pragma unroll
    for (int r = 0; r < R; ++r) {
        t.d[r] = make_uint4(INF, INF, INF, INF);
        if (ok && ((act >> r) & 1u)) t.d[r] = load_stream4(g.D + (int64_t)(r0 + r) * g.ld + c0);
    }
}

// Calls body(tile, c0, t) for every tile t of the rows' columns [0, n),
// c0 = 4 SWEEP_THREADS t + 4 thread-in-block: a work-group of SWEEP_THREADS
// threads spans SWEEP_THREADS / 64 column chunks of 256 per tile.
constexpr int SWEEP_THREADS = 512;
template <int R, class Body>
__device__ __forceinline__ void sweep_rows(const DevGraph &g, int32_t r0, uint32_t act, int32_t n, const int32_t *v1,
                                           const int32_t *v2, Body body) {
    const int32_t tiles = (n + 4 * SWEEP_THREADS - 1) / (4 * SWEEP_THREADS);
    int32_t c0 = threadIdx.x * 4;
    SweepTile<R> T;
    for (int32_t t = 0; t < tiles; ++t, c0 += 4 * SWEEP_THREADS) {
        sweep_load<R>(T, g, r0, act, c0, n, v1, v2);
        body(T, c0, t);
    }
}

// D[i][c0..c0+3] := min(D, t) over columns below n, stored only when
// something changed.
__device__ __forceinline__ void store_min_if_lower(const DevGraph &g, int32_t i, int32_t c0, uint4 x, uint4 t) {
    if (t.x < x.x || t.y < x.y || t.z < x.z || t.w < x.w) {
        x.x = min(x.x, t.x);
        x.y = min(x.y, t.y);
        x.z = min(x.z, t.z);
        x.w = min(x.w, t.w);
        *reinterpret_cast<uint4 *>(g.D + (int64_t)i * g.ld + c0) = x;
    }
}

// Theorem 3: D[i][j] = min(D[i][j], in[i] (+) out[j]) over the old
// slots.  Block = 1024 columns x 8 rows; a row with in[i] = INF cannot change.
// Every row's 16-byte load is issued (non-temporal: D is streamed once)
// before any row is tested, so a lane has 8 loads in flight; the few changed
// groups are stored after.
constexpr int RELAX_ROWS = 8;

__global__ __launch_bounds__(256) void k_add_relax(DevGraph g, const int32_t *__restrict__ in,
                                                   const int32_t *__restrict__ out) {
    const int n = g.n_slots;
    const int32_t c0 = blockIdx.x * 1024 + threadIdx.x * 4;
    const int32_t r0 = blockIdx.y * RELAX_ROWS;
    if (c0 >= n) return;
    uint4 o = *reinterpret_cast<const uint4 *>(out + c0);
    if (c0 + 1 >= n) o.y = INF;
    if (c0 + 2 >= n) o.z = INF;
    if (c0 + 3 >= n) o.w = INF;
    uint32_t a[RELAX_ROWS];
    uint4 d[RELAX_ROWS];
#pragma unroll
    for (int r = 0; r < RELAX_ROWS; ++r) {
        const int32_t i = r0 + r;
        a[r] = i < n ? (uint32_t)in[i] : INF;
        d[r] = make_uint4(0, 0, 0, 0);
        if (a[r] < INF) d[r] = load_stream4(g.D + (int64_t)i * g.ld + c0);
    }
#pragma unroll
    for (int r = 0; r < RELAX_ROWS; ++r) {
        if (a[r] >= INF) continue;
        const uint4 t = make_uint4(cat(a[r], o.x), cat(a[r], o.y), cat(a[r], o.z), cat(a[r], o.w));
        uint4 x = d[r];
        if (t.x < x.x || t.y < x.y || t.z < x.z || t.w < x.w) {
            x.x = min(x.x, t.x);
            x.y = min(x.y, t.y);
            x.z = min(x.z, t.z);
            x.w = min(x.w, t.w);
            *reinterpret_cast<uint4 *>(g.D + (int64_t)(r0 + r) * g.ld + c0) = x;
        }
    }
}

// ---- undirected graphs: sweeps over the upper triangle ----
// D of an undirected graph is symmetric, and so are an addition's
// relaxation (in = out) and a removal's mask: such a sweep reads only the
// tiles of 8 rows x 1024 columns that reach the diagonal or lie above it, and
// whatever it changes or flags at (i, j), j > i, it also changes or flags at
// (j, i).  Tiles in order of row group rg, then column tile bx from rg / 128
// (the tile holding column 8 rg) on.
constexpr int32_t UPPER_GROUPS_PER_TILE = 1024 / 8;

__host__ __device__ inline int64_t upper_tile_count(int32_t n) {
    const int32_t nbx = (n + 1023) >> 10, groups = (n + 7) >> 3;
    int64_t t = 0;
    for (int32_t q = 0; q < nbx; ++q) {
        const int32_t g0 = q * UPPER_GROUPS_PER_TILE, g1 = min(groups, g0 + UPPER_GROUPS_PER_TILE);
        if (g1 > g0) t += (int64_t)(g1 - g0) * (nbx - q);
    }
    return t;
}

__device__ __forceinline__ void upper_tile_of(int32_t n, int64_t b, int32_t &rg, int32_t &bx) {
    const int32_t nbx = (n + 1023) >> 10, groups = (n + 7) >> 3;
    rg = bx = 0;
    for (int32_t q = 0; q < nbx; ++q) {
        const int32_t g0 = q * UPPER_GROUPS_PER_TILE, g1 = min(groups, g0 + UPPER_GROUPS_PER_TILE);
        const int64_t cnt = g1 > g0 ? (int64_t)(g1 - g0) * (nbx - q) : 0;
        if (b < cnt) {
            rg = g0 + (int32_t)(b / (nbx - q));
            bx = q + (int32_t)(b % (nbx - q));
            return;
        }
        b -= cnt;
    }
}

// An undirected addition's relaxation over the upper triangle: (i, j), j > i,
// and its mirror (j, i) take min(D[i][j], out[i] (+) out[j]).  A lane's 4
// columns wholly above the diagonal are stored as one 16-byte store when they
// changed; a group that meets the diagonal stores its changed entries one by
// one, since its entries at or below the diagonal take mirrored values from
// other lanes.  Row and column p are rewritten by the next kernel.
__global__ __launch_bounds__(256) void k_add_relax_sym(DevGraph g, const int32_t *__restrict__ out) {
    const int n = g.n_slots;
    int32_t rg, bx;
    upper_tile_of(n, blockIdx.x, rg, bx);
    const int32_t c0 = bx * 1024 + threadIdx.x * 4;
    const int32_t r0 = rg * RELAX_ROWS;
    if (c0 >= n || c0 + 3 <= r0) return;  // no column of this lane lies above a row of the group
    const int64_t ld = g.ld;
    uint4 o = *reinterpret_cast<const uint4 *>(out + c0);
    if (c0 + 1 >= n) o.y = INF;
    if (c0 + 2 >= n) o.z = INF;
    if (c0 + 3 >= n) o.w = INF;
    uint32_t a[RELAX_ROWS];
    uint4 d[RELAX_ROWS];
#pragma unroll
    for (int r = 0; r < RELAX_ROWS; ++r) {
        const int32_t i = r0 + r;
        a[r] = i < n && c0 + 3 > i ? (uint32_t)out[i] : INF;
        d[r] = make_uint4(0, 0, 0, 0);
        if (a[r] < INF) d[r] = load_stream4(g.D + (int64_t)i * ld + c0);
    }
#pragma unroll
    for (int r = 0; r < RELAX_ROWS; ++r) {
        if (a[r] >= INF) continue;
        const int32_t i = r0 + r;
        const uint32_t t[4] = {cat(a[r], o.x), cat(a[r], o.y), cat(a[r], o.z), cat(a[r], o.w)};
        uint32_t x[4] = {d[r].x, d[r].y, d[r].z, d[r].w};
        uint32_t ch = 0;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            if (c0 + e > i && t[e] < x[e]) {
                x[e] = t[e];
                ch |= 1u << e;
            }
        }
        if (!ch) continue;
        if (c0 > i) {
            *reinterpret_cast<uint4 *>(g.D + (int64_t)i * ld + c0) = make_uint4(x[0], x[1], x[2], x[3]);
        } else {
#pragma unroll
            for (int e = 0; e < 4; ++e)
                if ((ch >> e) & 1u) g.D[(int64_t)i * ld + c0 + e] = (int32_t)x[e];
        }
#pragma unroll
        for (int e = 0; e < 4; ++e)
            if ((ch >> e) & 1u) g.D[(int64_t)(c0 + e) * ld + i] = (int32_t)x[e];
    }
}

void launch_add_relax(const DevGraph &g, const int32_t *in, const int32_t *out, hipStream_t s) {
    if (g.n_slots <= 0) return;
    if (g.undirected) {  // in == out
        k_add_relax_sym<<<(unsigned)upper_tile_count(g.n_slots), 256, 0, s>>>(g, out);
        return;
    }
    dim3 grid((g.n_slots + 1023) / 1024, (g.n_slots + RELAX_ROWS - 1) / RELAX_ROWS);
    k_add_relax<<<grid, 256, 0, s>>>(g, in, out);
}

// Write the new node's row and column of D and A (and A^T) and register it.
// The end of an addition, one launch (its parts are independent):
//   row and column p of D and A (and A^T) written, p registered (thread
//   s < n_slots), and the rows the relaxation could change (in[s] < INF)
//   counted for the update statistics, one atomic per block;
//   p's out-edge to y entered in y's light in-edge list (one wave per y).
__global__ __launch_bounds__(256) void k_add_finish(DevGraph g, int32_t p, int32_t new_id, int32_t rank,
                                                    int32_t *slot_of_rank, const int32_t *in, const int32_t *out,
                                                    const int32_t *wo, const int32_t *wi) {
    __shared__ uint32_t red[8];
    const int32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t ld = g.ld;
    int relaxed = 0;
    if (s == p) {
        g.D[(int64_t)p * ld + p] = 0;
        g.A[(int64_t)p * ld + p] = 0;
        if (!g.undirected) g.AT[(int64_t)p * ld + p] = 0;
        g.id_of_slot[p] = new_id;
        slot_of_rank[rank] = p;
    } else if (s < g.n_slots) {
        relaxed = (uint32_t)in[s] < INF;
        g.D[(int64_t)p * ld + s] = out[s];
        g.D[(int64_t)s * ld + p] = in[s];
        g.A[(int64_t)p * ld + s] = wo[s];
        g.A[(int64_t)s * ld + p] = wi[s];
        if (!g.undirected) {
            g.AT[(int64_t)s * ld + p] = wo[s];
            g.AT[(int64_t)p * ld + s] = wi[s];
        }
    }
    relaxed = block_sum256(relaxed, red);
    if (threadIdx.x == 0 && relaxed) atomicAdd(&g.ctl->rows_relaxed, relaxed);
    const int32_t y = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (y < g.n_slots && y != p && g.id_of_slot[y] >= 0) wave_list_insert(g, y, p, (uint32_t)wo[y]);
}

void launch_add_finish(const DevGraph &g, int32_t p, int32_t new_id, int32_t rank, int32_t *slot_of_rank,
                       const int32_t *in, const int32_t *out, const int32_t *wo, const int32_t *wi, hipStream_t s) {
    k_add_finish<<<(g.n_slots + 3) / 4, 256, 0, s>>>(g, p, new_id, rank, slot_of_rank, in, out, wo, wi);
}

// ---------------------------------------------------------------------------
// gathers, tombstones, bookkeeping
// ---------------------------------------------------------------------------

// The start of a removal: the per-update counters zeroed (thread 0 of block
// 0), column / row k of D gathered: colk[i] = D[i][k], rowk[j] = D[k][j],
// and the first mark_words words of the row marks zeroed (an undirected
// mask ORs its marks in).
__global__ void k_remove_begin(DevGraph g, int32_t k, int32_t *colk, int32_t *rowk, uint32_t *marks,
                               int32_t mark_words) {
    if (blockIdx.x == 0 && threadIdx.x == 0) reset_stats(g.ctl);
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    for (int32_t w = i; w < mark_words; w += gridDim.x * blockDim.x) marks[w] = 0u;
    if (i >= g.n_slots) return;
    const int32_t rk = g.D[(int64_t)k * g.ld + i];
    rowk[i] = rk;
    colk[i] = g.undirected ? rk : g.D[(int64_t)i * g.ld + k];  // D symmetric when undirected
}

void launch_remove_begin(const DevGraph &g, int32_t k, int32_t *colk, int32_t *rowk, uint8_t *marks, hipStream_t s) {
    if (g.n_slots <= 0) return;
    // marks: 256-byte aligned, (P / 8) rows of mark_pitch bytes, padded to 256
    const int32_t words = g.undirected ? (int32_t)(((int64_t)(g.n_slots + 7) / 8 * mark_pitch(g.P) + 3) / 4) : 0;
    k_remove_begin<<<(g.n_slots + 255) / 256, 256, 0, s>>>(g, k, colk, rowk, reinterpret_cast<uint32_t *>(marks),
                                                           words);
}

// The end of a removal, one launch (its parts are independent):
//   G - G_k: row and column k of D, A (and A^T) become INF, diagonal
//     included (thread s < n_slots);
//   k dropped from every light in-edge list, k's own list emptied, lists that
//     fall below half queued for a rebuild (one wave per list y);
//   the rank -> slot table without rank r (thread t < n_live - 1).
__global__ __launch_bounds__(256) void k_remove_finish(DevGraph g, int32_t k, int32_t *queue, const int32_t *rank_src,
                                                       int32_t *rank_dst, int32_t r, int32_t n_live,
                                                       const int32_t *partials, int32_t blocks) {
    __shared__ uint32_t red[8];
    if (blockIdx.x == 0) mask_finish_block<256>(g, partials, blocks, red);  // the recompute's statistics
    const int32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s < g.n_slots) {
        const int64_t ld = g.ld;
        const int32_t I = (int32_t)INF;
        g.D[(int64_t)k * ld + s] = I;
        g.D[(int64_t)s * ld + k] = I;
        g.A[(int64_t)k * ld + s] = I;
        g.A[(int64_t)s * ld + k] = I;
        if (!g.undirected) {
            g.AT[(int64_t)k * ld + s] = I;
            g.AT[(int64_t)s * ld + k] = I;
        }
        if (s == k) g.id_of_slot[k] = -1;
    }
    if (s < n_live - 1) rank_dst[s] = rank_src[s < r ? s : s + 1];
    const int32_t y = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (y >= g.n_slots) return;  // wave-uniform
    if (y == k) {
        g.nin[(int64_t)y * NIN_L + lane_id()] = make_int2(0, (int)INF);
        if (lane_id() == 0) { g.nin_cnt[y] = 0; g.nin_beta[y] = (int32_t)INF; }
        return;
    }
    const int before = g.nin_cnt[y];
    wave_list_purge(g, y, k);
    if (lane_id() == 0 && before >= NIN_L / 2 && before - 1 < NIN_L / 2 && (uint32_t)g.nin_beta[y] < INF &&
        g.id_of_slot[y] >= 0) {
        queue[atomicAdd(&g.ctl->short_count, 1)] = y;
    }
}

void launch_remove_finish(const DevGraph &g, int32_t k, int32_t *queue, const int32_t *rank_src, int32_t *rank_dst,
                          int32_t r, int32_t n_live, const int32_t *partials, int32_t blocks, hipStream_t s) {
    if (g.n_slots <= 0) return;
    k_remove_finish<<<(g.n_slots + 3) / 4, 256, 0, s>>>(g, k, queue, rank_src, rank_dst, r, n_live, partials, blocks);
}

// ---------------------------------------------------------------------------
// edge update (Section 3.3), decided on the device
// ---------------------------------------------------------------------------

// The decision (wave 0 of block 0: mode, old weight, the new weight in A,
// the index lists of v and u patched), after which block 0 rebuilds either
// list from the new weights if the patch left it short; and the gathers of
// columns u, v and rows u, v of D, which the decision does not touch, in one
// launch.  Every later step of the update sees the patched (or rebuilt)
// lists; any list that keeps the index invariant serves the recompute.
__global__ __launch_bounds__(256) void k_edge_begin(DevGraph g, int32_t su, int32_t sv, int32_t w, int32_t *colu,
                                                    int32_t *colv, int32_t *rowu, int32_t *rowv, uint32_t *marks,
                                                    int32_t mark_words) {
    __shared__ SelectShared sh;
    extern __shared__ uint32_t stage[];
    // an undirected increase's mask ORs its row marks in
    for (int32_t q = blockIdx.x * blockDim.x + threadIdx.x; q < mark_words; q += gridDim.x * blockDim.x) marks[q] = 0u;
    if (blockIdx.x == 0) {  // block-uniform
        if (threadIdx.x < 64) edge_begin_wave(g, su, sv, w);
        __syncthreads();
        nin_build_one(g, sv, 1, sh, stage);
        if (g.undirected) {
            __syncthreads();
            nin_build_one(g, su, 1, sh, stage);
        }
    }
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= g.n_slots) return;
    const int64_t ld = g.ld;
    const int32_t ru = g.D[(int64_t)su * ld + i], rv = g.D[(int64_t)sv * ld + i];
    rowu[i] = ru;
    rowv[i] = rv;
    // an undirected graph's D is symmetric: its columns are read as rows
    colu[i] = g.undirected ? ru : g.D[(int64_t)i * ld + su];
    colv[i] = g.undirected ? rv : g.D[(int64_t)i * ld + sv];
}

void launch_edge_begin(const DevGraph &g, int32_t su, int32_t sv, int32_t w, int32_t *colu, int32_t *colv,
                       int32_t *rowu, int32_t *rowv, uint8_t *marks, hipStream_t s) {
    const int32_t words = g.undirected ? (int32_t)(((int64_t)(g.n_slots + 7) / 8 * mark_pitch(g.P) + 3) / 4) : 0;
    k_edge_begin<<<(g.n_slots + 255) / 256, 256, nin_build_lds_bytes(g.P), s>>>(
        g, su, sv, w, colu, colv, rowu, rowv, reinterpret_cast<uint32_t *>(marks), words);
}

// Decrease of u -> v to w (< D[u][v]).  Inserting a relay node on the edge
// and applying Theorem 3 gives
//   D'[i][j] = min(D[i][j], D[i][u] (+) w (+) D[v][j])   (and v -> u if undirected).
// Only rows with D[i][u] (+) w < D[i][v] can change.  The column / row vectors
// were gathered before this launch, so in-place writes do not feed back.
// The rows r0 .. r0 + SWEEP_ROWS - 1 of one work-group.
__device__ __forceinline__ void dec_relax_rows(const DevGraph &g, const int32_t *__restrict__ colu,
                                               const int32_t *__restrict__ colv, const int32_t *__restrict__ rowu,
                                               const int32_t *__restrict__ rowv, int32_t w, int32_t r0) {
    const int n = g.n_slots;
    const uint32_t wn = (uint32_t)w;
    uint32_t x1[SWEEP_ROWS], x2[SWEEP_ROWS];
    uint32_t act = 0;
#pragma unroll
    for (int r = 0; r < SWEEP_ROWS; ++r) {
        const int32_t i = r0 + r;
        x1[r] = x2[r] = INF;
        if (i < n) {
            const uint32_t du = (uint32_t)colu[i], dv = (uint32_t)colv[i];
            if (cat(du, wn) < dv) x1[r] = cat(du, wn);
            if (g.undirected && cat(dv, wn) < du) x2[r] = cat(dv, wn);
            if (x1[r] < INF || x2[r] < INF) act |= 1u << r;
        }
    }
    if (act == 0) return;  // block-uniform
    if (threadIdx.x == 0) atomicAdd(&g.ctl->rows_relaxed, __popc(act));
    sweep_rows<SWEEP_ROWS>(g, r0, act, n, rowv, g.undirected ? rowu : nullptr,
                           [&](const SweepTile<SWEEP_ROWS> &T, int32_t c0, int32_t) {
        if (c0 >= n) return;
        const uint4 bv = T.v1, bu = T.v2;  // INF where absent or past n
#pragma unroll
        for (int r = 0; r < SWEEP_ROWS; ++r) {
            if (!((act >> r) & 1u)) continue;
            store_min_if_lower(g, r0 + r, c0, T.d[r],
                               make_uint4(min(cat(x1[r], bv.x), cat(x2[r], bu.x)), min(cat(x1[r], bv.y), cat(x2[r], bu.y)),
                                          min(cat(x1[r], bv.z), cat(x2[r], bu.z)), min(cat(x1[r], bv.w), cat(x2[r], bu.w))));
        }
    });
}


// ---------------------------------------------------------------------------
// mask + exact recompute (node removal, edge increase)
// ---------------------------------------------------------------------------
// One block per affected row i (blocks stride over rows).
//   1. Stream row i once, flag column j when a pair test holds
//        remove k:   D[i][k] (+) D[k][j] == D[i][j]          (Corollary 3)
//        increase:   D[i][u] (+) w_old (+) D[v][j] == D[i][j]  (and v -> u if undirected)
//      with j != i, D[i][j] < INF (j != k for a removal).  Unflagged entries
//      keep their value in G' (Theorem 4); flagged ones start at
//      INF in an LDS copy `cur` of the row, as does column k.
//   2. Recompute the flagged entries on G' by Bellman-Ford relaxation
//        cur[y] = min_x cur[x] (+) A'[x][y]
//      restricted to the flagged y.  The unflagged x already hold exact
//      values, so the fixed point is the exact row of G'.  Each y scans its
//      light in-edge list in ascending weight and stops when the weight
//      reaches cur[y]; a y whose value stays above its list bound beta takes
//      an exhaustive scan of its in-edges.  Sweeps repeat until nothing
//      changes.
//   3. Write the flagged entries back.
// Every value written is the length of a real walk in G' and the final row
// satisfies every edge inequality of G', so it equals SPD in G' exactly.

// LDS words: cur[P] | two flag bitmaps | list[LDS_LIST] | 64 scratch words.
size_t fused_lds_bytes(int32_t P) {
    return ((size_t)P + 2 * (size_t)((P + 31) / 32) + LDS_LIST + 64) * sizeof(uint32_t);
}

// Pass A, in two kernels.
//   detect: stream D in tiles of 8 rows x 1024 columns (the pair-test row
//     slice stays in registers, the 8 rows' loads are issued together) and
//     write the nonzero flag words (32 columns per word, assembled by 8 lanes
//     with DPP moves) into the bitmap, which is zero everywhere else: its
//     readers clear the words they used.  Each wavefront stores one byte of
//     row marks for its 8 rows x 256 columns (plain stores: no atomics and
//     no block barrier).
//   recompute: one wavefront per row with a mark.  The row's flagged columns
//     are read from the bitmap; the row of D itself is `cur`: flagged entries
//     (and column k of a removal) are set to INF and relaxed in place by
//     Bellman-Ford over the light in-edge index.  Rows with more than ROW_CAP
//     flags ("heavy") are left untouched and queued for pass B.
// OR of the 32-bit values of the 8 lanes of each aligned group of 8.
__device__ __forceinline__ uint32_t or8(uint32_t v) {
    v |= (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0xB1, 0xF, 0xF, false);   // quad_perm [1,0,3,2]
    v |= (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x4E, 0xF, 0xF, false);   // quad_perm [2,3,0,1]
    v |= (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x141, 0xF, 0xF, false);  // row_half_mirror
    return v;
}

// The mask of rows r0 .. r0 + SWEEP_ROWS - 1 (one work-group).  Each tile
// writes its nonzero flag words and, per wavefront, the byte of row marks of
// its 8 rows x 256 columns -- also when nothing is flagged, since the marks
// are rewritten by every detection.
template <int MODE>
__device__ __forceinline__ void mask_detect_rows(const DevGraph &g, const FusedArgs &fa, uint32_t w_old, int32_t r0) {
    static_assert(SWEEP_ROWS == 8, "a byte of row marks covers 8 rows");
    const int n = g.n_slots;
    const int lane = lane_id();
    const int64_t nwp = (g.P + 31) / 32;
    const int32_t rg = r0 / SWEEP_ROWS;
    const int kx = MODE == FUSED_REMOVE ? fa.k : -1;
    uint32_t a1[SWEEP_ROWS], a2[SWEEP_ROWS];
    uint32_t act = 0;
#pragma unroll
    for (int r = 0; r < SWEEP_ROWS; ++r) {
        const int32_t i = r0 + r;
        a1[r] = a2[r] = 0x80000000u;  // disabled: a (+) v exceeds every finite entry
        if (i < n) {
            const RowTests rt = row_tests(g, fa, i, w_old);
            if (rt.t1) a1[r] = rt.a1;
            if (rt.t2) a2[r] = rt.a2;
            if (rt.t1 || rt.t2) act |= 1u << r;
        }
    }
    sweep_rows<SWEEP_ROWS>(g, r0, act, n, fa.row1, MODE == FUSED_INCREASE ? fa.row2 : nullptr,
                           [&](const SweepTile<SWEEP_ROWS> &T, int32_t c0, int32_t t) {
        const uint32_t w1[4] = {T.v1.x, T.v1.y, T.v1.z, T.v1.w};
        const uint32_t w2[4] = {T.v2.x, T.v2.y, T.v2.z, T.v2.w};
        uint32_t row_mask = 0;  // rows of this wavefront's 8 x 256 tile holding a flag (wave-uniform)
#pragma unroll
        for (int r = 0; r < SWEEP_ROWS; ++r) {
            if (!((act >> r) & 1u)) continue;  // block-uniform
            const int32_t i = r0 + r;
            const uint32_t dv[4] = {T.d[r].x, T.d[r].y, T.d[r].z, T.d[r].w};
            uint32_t bits = 0;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int32_t j = c0 + e;
                bool f = cat(a1[r], w1[e]) == dv[e];
                if (MODE == FUSED_INCREASE) f = f || (cat(a2[r], w2[e]) == dv[e]);
                f = f && dv[e] < INF && j != i && j != kx && j < n;
                bits |= (uint32_t)f << e;
            }
            const uint32_t word = or8(bits << ((lane & 7) * 4));
            if ((lane & 7) == 0 && c0 < n && word != 0) fa.flag_bits[(int64_t)i * nwp + (c0 >> 5)] = word;
            if (__ballot(bits != 0) != 0) row_mask |= 1u << r;
        }
        const int32_t chunk = c0 >> 8;  // this wavefront's 256 columns
        if (lane == 0 && chunk * 256 < n) fa.marks[(int64_t)rg * fa.mark_pitch + chunk] = (uint8_t)row_mask;
    });
}

// The removal mask over one tile of 8 rows x 1024 columns (one work-group per
// tile): the 8 rows' loads issued together before any test.
constexpr int DETECT_ROWS = 8;
template <int MODE>
__device__ __forceinline__ void mask_detect_tile(const DevGraph &g, const FusedArgs &fa, uint32_t w_old, int32_t rg) {
    const int n = g.n_slots;
    const int lane = lane_id();
    const int32_t c0 = blockIdx.x * 1024 + threadIdx.x * 4;
    const int32_t r0 = rg * DETECT_ROWS;
    const int64_t nwp = (g.P + 31) / 32;
    uint4 v1 = make_uint4(0, 0, 0, 0), v2 = v1;
    if (c0 < n) {
        v1 = *reinterpret_cast<const uint4 *>(fa.row1 + c0);
        if (MODE == FUSED_INCREASE) v2 = *reinterpret_cast<const uint4 *>(fa.row2 + c0);
    }
    const uint32_t w1[4] = {v1.x, v1.y, v1.z, v1.w};
    const uint32_t w2[4] = {v2.x, v2.y, v2.z, v2.w};
    const int kx = MODE == FUSED_REMOVE ? fa.k : -1;
    uint32_t row_mask = 0;  // rows of this wavefront's 8 x 256 tile holding a flag (wave-uniform)
    uint4 d[DETECT_ROWS];
    uint32_t a1[DETECT_ROWS], a2[DETECT_ROWS];
    bool tested[DETECT_ROWS];
#pragma unroll
    for (int r = 0; r < DETECT_ROWS; ++r) {
        const int32_t i = r0 + r;
        d[r] = make_uint4(INF, INF, INF, INF);
        a1[r] = a2[r] = 0x80000000u;  // disabled: a (+) v exceeds every finite entry
        tested[r] = false;
        if (i < n) {
            const RowTests rt = row_tests(g, fa, i, w_old);
            if (rt.t1) a1[r] = rt.a1;
            if (rt.t2) a2[r] = rt.a2;
            tested[r] = rt.t1 || rt.t2;
            if (tested[r] && c0 < n) d[r] = load_stream4(g.D + (int64_t)i * g.ld + c0);
        }
    }
#pragma unroll
    for (int r = 0; r < DETECT_ROWS; ++r) {
        if (!tested[r]) continue;  // block-uniform
        const int32_t i = r0 + r;
        const uint32_t dv[4] = {d[r].x, d[r].y, d[r].z, d[r].w};
        uint32_t bits = 0;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int32_t j = c0 + e;
            bool f = cat(a1[r], w1[e]) == dv[e];
            if (MODE == FUSED_INCREASE) f = f || (cat(a2[r], w2[e]) == dv[e]);
            f = f && dv[e] < INF && j != i && j != kx;
            bits |= (uint32_t)f << e;
        }
        const uint32_t word = or8(bits << ((lane & 7) * 4));
        if ((lane & 7) == 0 && c0 < n && word != 0) fa.flag_bits[(int64_t)i * nwp + (c0 >> 5)] = word;
        if (__ballot(bits != 0) != 0) row_mask |= 1u << r;
    }
    const int32_t chunk = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (lane == 0 && chunk * 256 < n) fa.marks[(int64_t)rg * fa.mark_pitch + chunk] = (uint8_t)row_mask;
}

__global__ __launch_bounds__(256) void k_mask_detect(DevGraph g, FusedArgs fa) {
    mask_detect_tile<FUSED_REMOVE>(g, fa, 0u, blockIdx.y);
}

// OR bits into the row-mark byte of row group grp and chunk (the marks are
// zeroed by the update's first kernel).
__device__ __forceinline__ void mark_or(const FusedArgs &fa, int32_t grp, int32_t chunk, uint32_t bits) {
    const int64_t off = (int64_t)grp * fa.mark_pitch + chunk;
    atomicOr(reinterpret_cast<uint32_t *>(fa.marks + (off & ~(int64_t)3)), bits << (8 * (off & 3)));
}

// An undirected removal's mask over one upper tile (see upper_tile_of): the
// pairs (i, j), j > i, tested as in mask_detect_tile, each flag also set at
// (j, i).  A row's flag word that holds its diagonal also takes mirrored bits
// and is ORed in; its words further right take none and are stored.  Each
// lane ORs its columns' mirrored bits (8 rows: a byte of row j's word that
// holds columns r0 .. r0 + 7) and their marks in.
__global__ __launch_bounds__(256) void k_mask_detect_sym(DevGraph g, FusedArgs fa) {
    const int n = g.n_slots;
    const int lane = lane_id();
    int32_t rg, bx;
    upper_tile_of(n, blockIdx.x, rg, bx);
    const int32_t c0 = bx * 1024 + threadIdx.x * 4;
    const int32_t r0 = rg * DETECT_ROWS;
    const int64_t nwp = (g.P + 31) / 32;
    uint4 v1 = make_uint4(0, 0, 0, 0);
    if (c0 < n) v1 = *reinterpret_cast<const uint4 *>(fa.row1 + c0);
    const uint32_t w1[4] = {v1.x, v1.y, v1.z, v1.w};
    const int kx = fa.k;
    uint32_t row_mask = 0;         // rows of this wavefront's 8 x 256 tile holding a flag (wave-uniform)
    uint32_t mir[4] = {0, 0, 0, 0};  // per column of the lane: bit r = flag of row r0 + r
    uint4 d[DETECT_ROWS];
    uint32_t a1[DETECT_ROWS];
    bool tested[DETECT_ROWS];
#pragma unroll
    for (int r = 0; r < DETECT_ROWS; ++r) {
        const int32_t i = r0 + r;
        d[r] = make_uint4(INF, INF, INF, INF);
        a1[r] = 0x80000000u;  // disabled: a (+) v exceeds every finite entry
        tested[r] = false;
        if (i < n) {
            const RowTests rt = row_tests(g, fa, i, 0u);
            if (rt.t1) a1[r] = rt.a1;
            tested[r] = rt.t1;
            if (tested[r] && c0 < n && c0 + 3 > i) d[r] = load_stream4(g.D + (int64_t)i * g.ld + c0);
        }
    }
#pragma unroll
    for (int r = 0; r < DETECT_ROWS; ++r) {
        if (!tested[r]) continue;  // block-uniform
        const int32_t i = r0 + r;
        const uint32_t dv[4] = {d[r].x, d[r].y, d[r].z, d[r].w};
        uint32_t bits = 0;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int32_t j = c0 + e;
            const bool f = cat(a1[r], w1[e]) == dv[e] && dv[e] < INF && j > i && j != kx;
            bits |= (uint32_t)f << e;
            mir[e] |= (uint32_t)f << r;
        }
        const uint32_t word = or8(bits << ((lane & 7) * 4));
        if ((lane & 7) == 0 && c0 < n && word != 0) {
            uint32_t *wp = fa.flag_bits + (int64_t)i * nwp + (c0 >> 5);
            if ((c0 >> 5) == (i >> 5)) atomicOr(wp, word);
            else *wp = word;
        }
        if (__ballot(bits != 0) != 0) row_mask |= 1u << r;
    }
    if (lane == 0 && row_mask) mark_or(fa, rg, bx * 4 + (threadIdx.x >> 6), row_mask);
    uint32_t mbits = 0;  // the lane's 4 columns share a row group
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        if (!mir[e]) continue;
        const int32_t j = c0 + e;
        atomicOr(fa.flag_bits + (int64_t)j * nwp + (r0 >> 5), mir[e] << (r0 & 31));
        mbits |= 1u << (j & 7);
    }
    if (mbits) mark_or(fa, c0 >> 3, r0 >> 8, mbits);
}

// |F| and Phi of a removal's (or a tight increase's) mask, counted without
// writing it (a route that needs no flags still reports them, and Algorithm
// 5's cost test reads Phi).
__global__ __launch_bounds__(SWEEP_THREADS) void k_mask_count(DevGraph g, FusedArgs fa) {
    __shared__ uint32_t s_cnt, s_rows;
    const int n = g.n_slots;
    const int32_t r0 = blockIdx.x * SWEEP_ROWS;
    const bool inc = fa.mode == FUSED_INCREASE;
    const uint32_t w_old = inc ? (uint32_t)g.ctl->w_old : 0u;
    const int32_t kx = inc ? -1 : fa.k;
    uint32_t a1[SWEEP_ROWS], a2[SWEEP_ROWS];
    uint32_t act = 0;
#pragma unroll
    for (int r = 0; r < SWEEP_ROWS; ++r) {
        a1[r] = a2[r] = 0x80000000u;
        if (r0 + r < n) {
            const RowTests rt = row_tests(g, fa, r0 + r, w_old);
            if (rt.t1) a1[r] = rt.a1;
            if (rt.t2) a2[r] = rt.a2;
            if (rt.t1 || rt.t2) act |= 1u << r;
        }
    }
    if (act == 0) return;  // block-uniform
    if (threadIdx.x == 0) s_cnt = s_rows = 0;
    __syncthreads();
    uint32_t cnt = 0, rows = 0;
    sweep_rows<SWEEP_ROWS>(g, r0, act, n, fa.row1, inc ? fa.row2 : nullptr,
                           [&](const SweepTile<SWEEP_ROWS> &T, int32_t c0, int32_t) {
        const uint32_t w1[4] = {T.v1.x, T.v1.y, T.v1.z, T.v1.w};
        const uint32_t w2[4] = {T.v2.x, T.v2.y, T.v2.z, T.v2.w};
#pragma unroll
        for (int r = 0; r < SWEEP_ROWS; ++r) {
            if (!((act >> r) & 1u)) continue;
            const uint32_t dv[4] = {T.d[r].x, T.d[r].y, T.d[r].z, T.d[r].w};
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int32_t j = c0 + e;
                const bool f = (cat(a1[r], w1[e]) == dv[e] || cat(a2[r], w2[e]) == dv[e]) && dv[e] < INF &&
                               j != r0 + r && j != kx && j < n;
                cnt += f;
                rows |= (uint32_t)f << r;
            }
        }
    });
    if (cnt) atomicAdd(&s_cnt, cnt);
    if (rows) atomicOr(&s_rows, rows);
    __syncthreads();
    if (threadIdx.x == 0 && s_cnt) {
        atomicAdd(&g.ctl->flagged, (unsigned long long)s_cnt);
        atomicAdd(&g.ctl->rows, __popc(s_rows));
    }
}

// A tight increase's mask on an undirected graph (the rows r0 .. r0 + 7 of
// one work-group): both pair tests of mask_detect_rows on the pairs (i, j),
// j > i, each flag also set at (j, i) -- the mask is symmetric, its second
// test being the first read from the other end.  The walk starts at the tile
// that holds column r0; flag words and marks as in k_mask_detect_sym (the
// marks were zeroed by k_edge_begin).
__device__ __forceinline__ void inc_mask_rows_sym(const DevGraph &g, const FusedArgs &fa, uint32_t w_old, int32_t r0) {
    const int n = g.n_slots;
    const int lane = lane_id();
    const int64_t nwp = (g.P + 31) / 32;
    const int32_t rg = r0 / SWEEP_ROWS;
    uint32_t a1[SWEEP_ROWS], a2[SWEEP_ROWS];
    uint32_t act = 0;
#pragma unroll
    for (int r = 0; r < SWEEP_ROWS; ++r) {
        const int32_t i = r0 + r;
        a1[r] = a2[r] = 0x80000000u;  // disabled: a (+) v exceeds every finite entry
        if (i < n) {
            const RowTests rt = row_tests(g, fa, i, w_old);
            if (rt.t1) a1[r] = rt.a1;
            if (rt.t2) a2[r] = rt.a2;
            if (rt.t1 || rt.t2) act |= 1u << r;
        }
    }
    if (act == 0) return;  // block-uniform
    constexpr int32_t span = 4 * SWEEP_THREADS;
    const int32_t tiles = (n + span - 1) / span;
    int32_t c0 = (r0 / span) * span + threadIdx.x * 4;
    SweepTile<SWEEP_ROWS> T;
    for (int32_t t = r0 / span; t < tiles; ++t, c0 += span) {
        sweep_load<SWEEP_ROWS>(T, g, r0, act, c0, n, fa.row1, fa.row2);
        const uint32_t w1[4] = {T.v1.x, T.v1.y, T.v1.z, T.v1.w};
        const uint32_t w2[4] = {T.v2.x, T.v2.y, T.v2.z, T.v2.w};
        uint32_t row_mask = 0;           // rows of this wavefront's 8 x 256 tile holding a flag (wave-uniform)
        uint32_t mir[4] = {0, 0, 0, 0};  // per column of the lane: bit r = flag of row r0 + r
#pragma unroll
        for (int r = 0; r < SWEEP_ROWS; ++r) {
            if (!((act >> r) & 1u)) continue;  // block-uniform
            const int32_t i = r0 + r;
            const uint32_t dv[4] = {T.d[r].x, T.d[r].y, T.d[r].z, T.d[r].w};
            uint32_t bits = 0;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int32_t j = c0 + e;
                const bool f = (cat(a1[r], w1[e]) == dv[e] || cat(a2[r], w2[e]) == dv[e]) && dv[e] < INF && j > i &&
                               j < n;
                bits |= (uint32_t)f << e;
                mir[e] |= (uint32_t)f << r;
            }
            const uint32_t word = or8(bits << ((lane & 7) * 4));
            if ((lane & 7) == 0 && c0 < n && word != 0) {
                uint32_t *wp = fa.flag_bits + (int64_t)i * nwp + (c0 >> 5);
                if ((c0 >> 5) == (i >> 5)) atomicOr(wp, word);
                else *wp = word;
            }
            if (__ballot(bits != 0) != 0) row_mask |= 1u << r;
        }
        if (lane == 0 && row_mask) mark_or(fa, rg, c0 >> 8, row_mask);
        uint32_t mbits = 0;  // the lane's 4 columns share a row group
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            if (!mir[e]) continue;
            const int32_t j = c0 + e;
            atomicOr(fa.flag_bits + (int64_t)j * nwp + (r0 >> 5), mir[e] << (r0 & 31));
            mbits |= 1u << (j & 7);
        }
        if (mbits) mark_or(fa, c0 >> 3, r0 >> 8, mbits);
    }
}

// The edge update's sweep, chosen on the device: the relaxation of a decrease
// (colu, colv, rowu, rowv = fa.col1, col2, row2, row1) or the mask of a tight
// increase; nothing for a no-op.  One work-group per SWEEP_ROWS rows (the
// grid of a no-op launch is n / SWEEP_ROWS work-groups that return at once).
__global__ __launch_bounds__(SWEEP_THREADS) void k_edge_sweep(DevGraph g, FusedArgs fa, int32_t w) {
    const int32_t mode = g.ctl->edge_mode;
    if (mode == EDGE_NOOP) return;
    const int32_t r0 = blockIdx.x * SWEEP_ROWS;
    if (mode == EDGE_DECREASE) dec_relax_rows(g, fa.col1, fa.col2, fa.row2, fa.row1, w, r0);
    else if (g.undirected) inc_mask_rows_sym(g, fa, (uint32_t)g.ctl->w_old, r0);
    else mask_detect_rows<FUSED_INCREASE>(g, fa, (uint32_t)g.ctl->w_old, r0);
}

// Does row i hold a flag?  (The OR of its group's marks, read by one wave.)
__device__ __forceinline__ bool row_marked(const FusedArgs &fa, int32_t n, int32_t i) {
    const uint8_t *m = fa.marks + (int64_t)(i >> 3) * fa.mark_pitch;
    const int32_t chunks = (n + 255) >> 8;
    uint32_t v = 0;
    for (int32_t c = lane_id(); c < chunks; c += 64) v |= m[c];
    return __ballot((v >> (i & 7)) & 1u) != 0;
}

// Phi of the pending mask (Algorithm 5's cost needs it before the recompute).
__global__ __launch_bounds__(256) void k_count_flag_rows(DevGraph g, FusedArgs fa) {
    __shared__ uint32_t red[8];
    const int32_t chunks = (g.n_slots + 255) >> 8;
    int c = 0;
    for (int32_t grp = threadIdx.x; grp < (g.n_slots + 7) / 8; grp += 256) {
        const uint8_t *m = fa.marks + (int64_t)grp * fa.mark_pitch;
        uint32_t v = 0;
        for (int32_t q = 0; q < chunks; ++q) v |= m[q];
        c += __popc(v);
    }
    c = block_sum256(c, red);
    if (threadIdx.x == 0) g.ctl->rows = c;
}

// reset_only: only clear the flagged rows' words (after a cold fallback).
// A row's flag words are cleared once read, except those of an undirected
// heavy row, which the heavy-row pass reads (and clears) later.
__global__ __launch_bounds__(64 * RECOMPUTE_WAVES, 5) void k_recompute_rows(DevGraph g, FusedArgs fa, int32_t reset_only) {
    __shared__ int32_t lists[RECOMPUTE_WAVES][ROW_CAP];
    __shared__ int32_t fsls[RECOMPUTE_WAVES][ROW_CAP];
    __shared__ int32_t olds[RECOMPUTE_WAVES][ROW_CAP];
    __shared__ int32_t stat[RECOMPUTE_WAVES][RECOMPUTE_STATS];
    __shared__ uint32_t dense[RECOMPUTE_WAVES][ROW_CAP * ROW_CAP];  // light in-edges among a row's flagged columns
    __shared__ uint32_t vals[RECOMPUTE_WAVES][ROW_CAP];
    __shared__ int32_t fkeys[RECOMPUTE_WAVES][FSET];
    __shared__ int32_t fpos[RECOMPUTE_WAVES][FSET];
    const int lane = lane_id(), wv = threadIdx.x >> 6;
    int32_t *list = lists[wv];
    int32_t *fsl = fsls[wv];
    int32_t *old = olds[wv];
    const int n = g.n_slots;
    const int nw = (n + 31) / 32;
    const int64_t nwp = (g.P + 31) / 32;
    int my_rows = 0, my_fs = 0, my_sweeps = 0, my_flagged = 0, my_changed = 0, my_rows_changed = 0;
    const bool active = !(fa.mode == FUSED_INCREASE && g.ctl->edge_mode != EDGE_INCREASE);
    const uint32_t w_old = active && fa.mode == FUSED_INCREASE ? (uint32_t)g.ctl->w_old : 0u;
    for (int32_t i = blockIdx.x * RECOMPUTE_WAVES + wv; active && i < n; i += gridDim.x * RECOMPUTE_WAVES) {
        if (!row_marked(fa, n, i)) continue;
        ++my_rows;
        // flagged columns of row i -> list (at most ROW_CAP kept)
        uint32_t *fw = fa.flag_bits + (int64_t)i * nwp;
        int cnt = 0;
        uint32_t wd[8] = {0, 0, 0, 0, 0, 0, 0, 0};  // the row's words when they fit one pass (nw <= 512)
        for (int b = 0; b < nw; b += 512) {  // wave-uniform; 8 words per lane in flight
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
            if (!reset_only && cnt + __shfl(incl, 63) <= ROW_CAP) {
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    uint32_t bits = wd[q];
                    while (bits) {
                        const int bt = __ffs(bits) - 1;
                        bits &= bits - 1;
                        list[pos++] = (b + q * 64 + lane) * 32 + bt;
                    }
                }
            }
            cnt += __shfl(incl, 63);
        }
        my_flagged += cnt;
        if (reset_only || cnt <= ROW_CAP || !g.undirected) {
            if (nw <= 512) {
#pragma unroll
                for (int q = 0; q < 8; ++q)
                    if (wd[q]) fw[q * 64 + lane] = 0u;
            } else {
                for (int w = lane; w < nw; w += 64)
                    if (fw[w]) fw[w] = 0u;
            }
        }
        if (reset_only) continue;
        if (cnt > ROW_CAP) {
            if (lane == 0) {
                fa.heavy_epoch[i] = fa.epoch;
                fa.heavy_rows[atomicAdd(&g.ctl->heavy_count, 1)] = i;
            }
            continue;
        }
        int32_t *Drow = g.D + (int64_t)i * g.ld;
        if (fa.mode == FUSED_REMOVE && lane == 0) Drow[fa.k] = (int32_t)INF;
        __threadfence_block();
        int sweeps = 0;
        const RowTests rt = row_tests(g, fa, i, w_old);
        const uint32_t v = light_row(g, fa, rt, Drow, list, cnt, fsl, old, vals[wv], fkeys[wv], fpos[wv], dense[wv],
                                     sweeps, my_fs);
        my_sweeps = max(my_sweeps, sweeps);
        // the refined set: flagged entries whose distance went up
        const int ch = wave_sum(lane < cnt && v != (uint32_t)old[lane]);
        my_changed += ch;
        my_rows_changed += ch > 0;
        // undirected: D' is symmetric and so is the mask, so the final
        // entries of row i are also those of column i.  A heavy row j takes
        // its entry (j, i) from here; a light row j computes the same value
        // itself, and any interleaving of the two exact writes is harmless.
        if (lane < cnt) {
            const int32_t y = list[lane];
            Drow[y] = (int32_t)v;
            if (g.undirected) g.D[(int64_t)y * g.ld + i] = (int32_t)v;
        }
    }
    // statistics: one partial per work-group, summed by the update's next kernel
    if (lane == 0) {
        stat[wv][0] = my_rows;
        stat[wv][1] = my_flagged;
        stat[wv][2] = my_fs;
        stat[wv][3] = my_sweeps;
        stat[wv][4] = my_changed;
        stat[wv][5] = my_rows_changed;
    }
    __syncthreads();
    if (threadIdx.x < RECOMPUTE_STATS) {
        const int q = threadIdx.x;
        int v = stat[0][q];
#pragma unroll
        for (int w = 1; w < RECOMPUTE_WAVES; ++w) v = q == 3 ? max(v, stat[w][q]) : v + stat[w][q];
        fa.partials[blockIdx.x * RECOMPUTE_STATS + q] = v;
    }
}

// After the recompute: sum the recompute work-groups' statistics into the
// control block (one work-group of NT threads).
template <int NT>
__device__ __forceinline__ void mask_finish_block(const DevGraph &g, const int32_t *partials, int32_t blocks,
                                                  uint32_t *red) {
    int rows = 0, fs = 0, flagged = 0, changed = 0, rows_changed = 0;
    uint32_t sw = 0;
    // the heavy-row pass's (changed, rows changed) per work-group follow the
    // recompute's partials; blocks < 0 means it did not run (-blocks groups)
    const bool heavy = blocks > 0;
    if (blocks < 0) blocks = -blocks;
    if (heavy)
        for (int b = threadIdx.x; b < FUSED_GRID; b += NT) {
            const int32_t *hb = partials + (int64_t)RECOMPUTE_BLOCKS * RECOMPUTE_STATS + 2 * b;
            changed += hb[0];
            rows_changed += hb[1];
        }
    for (int b = threadIdx.x; b < blocks; b += NT) {
        const int32_t *pb = partials + (int64_t)b * RECOMPUTE_STATS;
        rows += pb[0];
        flagged += pb[1];
        fs += pb[2];
        sw = max(sw, (uint32_t)pb[3]);
        changed += pb[4];
        rows_changed += pb[5];
    }
    rows = block_sum<NT>(rows, red);
    flagged = block_sum<NT>(flagged, red);
    fs = block_sum<NT>(fs, red);
    changed = block_sum<NT>(changed, red);
    rows_changed = block_sum<NT>(rows_changed, red);
    sw = ~block_min<NT>(~sw, red);
    if (threadIdx.x == 0) {
        g.ctl->rows += rows;
        g.ctl->flagged += (unsigned long long)flagged;
        g.ctl->full_scans += fs;
        g.ctl->changed += (unsigned long long)changed;
        g.ctl->rows_changed += rows_changed;
        atomicMax(&g.ctl->sweeps, (int32_t)sw);
    }
}


// Pass B: the heavy rows, one block each with the row in LDS.
//   undirected: every flagged (i, j) whose row j was light already holds its
//   final value (written by pass A from D'[j][i]); the heavy-heavy entries
//   are recomputed by Bellman-Ford against the now exact remainder of the
//   row.
//   directed: every flagged entry is recomputed by Bellman-Ford.
// Counts the changed pairs among row i's flagged entries (list[0..cnt)),
// whose final values are cur[], and adds them to my_changed /
// my_rows_changed (block-uniform).  One entry per thread at a time, so that
// the old values' loads of a dense flag word are not one thread's chain.
__device__ __forceinline__ void heavy_count_changed(const FusedArgs &fa, const RowTests &rt, const uint32_t *cur,
                                                    const int32_t *list, int cnt, uint32_t *red, int &my_changed,
                                                    int &my_rows_changed) {
    int ch = 0;
    for (int e = threadIdx.x; e < cnt; e += FUSED_THREADS) {
        const int32_t y = list[e];
        ch += cur[y] != flagged_old(fa, rt, y);
    }
    ch = block_sum<FUSED_THREADS>(ch, red);
    my_changed += ch;
    my_rows_changed += ch > 0;
}

__device__ __forceinline__ void fused_heavy_body(const DevGraph &g, const FusedArgs &fa, uint32_t *sm) {
    FusedShared sh = fused_shared(g, sm);
    const int n = g.n_slots;
    const int nw = (n + 31) >> 5;
    const int tid = threadIdx.x;
    // this work-group's part of the refined-set statistics (summed with the
    // recompute's partials by the update's next kernel)
    int32_t *hp = fa.partials + (int64_t)RECOMPUTE_BLOCKS * RECOMPUTE_STATS + 2 * blockIdx.x;
    int my_changed = 0, my_rows_changed = 0;
    if (tid == 0) hp[0] = hp[1] = 0;
    uint32_t w_old = 0;
    if (fa.mode == FUSED_INCREASE) {
        if (g.ctl->edge_mode != EDGE_INCREASE) return;
        w_old = (uint32_t)g.ctl->w_old;
    }
    const int count = g.ctl->heavy_count;
    const int fill = g.undirected ? 1 : 0;
    int32_t *glist = fa.scratch + (int64_t)blockIdx.x * 2 * g.P;
    int32_t *fsl = glist + g.P;
    int my_fs = 0, my_sweeps = 0;
    if (g.undirected) {
        if (blockIdx.x >= count) return;
        const int64_t nwp = (g.P + 31) / 32;
        // bitmap of the heavy rows (sh.fl), built once per work-group
        for (int w = tid; w < nw; w += FUSED_THREADS) sh.fl[w] = 0;
        __syncthreads();
        for (int q = tid; q < count; q += FUSED_THREADS) {
            const int32_t r = fa.heavy_rows[q];
            atomicOr(&sh.fl[r >> 5], 1u << (r & 31));
        }
        __syncthreads();
        for (int idx = blockIdx.x; idx < count; idx += gridDim.x) {
            const int32_t i = fa.heavy_rows[idx];
            const RowTests rt = row_tests(g, fa, i, w_old);
            int32_t *Drow = g.D + (int64_t)i * g.ld;
            for (int32_t c = tid * 4; c < n; c += FUSED_THREADS * 4)
                *reinterpret_cast<uint4 *>(sh.cur + c) = *reinterpret_cast<const uint4 *>(Drow + c);
            uint32_t *fw = fa.flag_bits + (int64_t)i * nwp;
            for (int w = tid; w < nw; w += FUSED_THREADS) sh.fl2[w] = fw[w] & sh.fl[w];
            __syncthreads();
            const int todo = compact_bits(sh.fl2, nw, glist, sh.red);
            for (int e = tid; e < todo; e += FUSED_THREADS) sh.cur[glist[e]] = INF;
            if (fa.mode == FUSED_REMOVE && tid == 0) sh.cur[fa.k] = INF;
            int sweeps = 0;
            if (todo > 0) row_bellman_ford(g, sh, glist, todo, fsl, sweeps, my_fs);
            __syncthreads();
            for (int e = tid; e < todo; e += FUSED_THREADS) {
                const int32_t y = glist[e];
                Drow[y] = (int32_t)sh.cur[y];
            }
            if (tid == 0) my_sweeps = max(my_sweeps, sweeps);
            __syncthreads();
            // cur holds every final entry of the row (the light-row entries
            // came in mirrored); count the changed ones over all the row's
            // flags, then clear its words: the bitmap is left clear
            for (int w = tid; w < nw; w += FUSED_THREADS) sh.fl2[w] = fw[w];
            __syncthreads();
            const int all = compact_bits(sh.fl2, nw, glist, sh.red);
            heavy_count_changed(fa, rt, sh.cur, glist, all, sh.red, my_changed, my_rows_changed);
            for (int w = tid; w < nw; w += FUSED_THREADS)
                if (sh.fl2[w]) fw[w] = 0u;
            __syncthreads();
        }
        if (tid == 0 && my_fs) atomicAdd(&g.ctl->full_scans, my_fs);
        if (tid == 0 && my_sweeps) atomicMax(&g.ctl->sweeps, my_sweeps);
        if (tid == 0) {
            hp[0] = my_changed;
            hp[1] = my_rows_changed;
        }
        return;
    }
    for (int idx = blockIdx.x; idx < count; idx += gridDim.x) {
        const int32_t i = fa.heavy_rows[idx];
        const RowTests rt = row_tests(g, fa, i, w_old);
        block_sum<FUSED_THREADS>(mask_row(g, fa, i, rt, sh, true, fill), sh.red);
        const int todo = compact_bits(fill ? sh.fl2 : sh.fl, nw, glist, sh.red);
        int sweeps = 0;
        if (todo > 0) row_bellman_ford(g, sh, glist, todo, fsl, sweeps, my_fs);
        const int all = fill ? compact_bits(sh.fl, nw, glist, sh.red) : todo;
        int32_t *Drow = g.D + (int64_t)i * g.ld;
        for (int e = tid; e < all; e += FUSED_THREADS) {
            const int32_t y = glist[e];
            Drow[y] = (int32_t)sh.cur[y];
        }
        if (tid == 0) my_sweeps = max(my_sweeps, sweeps);
        __syncthreads();
        heavy_count_changed(fa, rt, sh.cur, glist, all, sh.red, my_changed, my_rows_changed);
        __syncthreads();
    }
    if (tid == 0 && my_fs) atomicAdd(&g.ctl->full_scans, my_fs);
    if (tid == 0 && my_sweeps) atomicMax(&g.ctl->sweeps, my_sweeps);
    if (tid == 0) {
        hp[0] = my_changed;
        hp[1] = my_rows_changed;
    }
}

__global__ __launch_bounds__(FUSED_THREADS) void k_fused_heavy(DevGraph g, FusedArgs fa) {
    extern __shared__ uint32_t sm[];
    fused_heavy_body(g, fa, sm);
}

void launch_mask_detect(const DevGraph &g, const FusedArgs &fa, hipStream_t s) {
    if (g.n_slots <= 0) return;
    if (g.undirected) {
        k_mask_detect_sym<<<(unsigned)upper_tile_count(g.n_slots), 256, 0, s>>>(g, fa);
        return;
    }
    dim3 grid((g.n_slots + 1023) / 1024, (g.n_slots + DETECT_ROWS - 1) / DETECT_ROWS);
    k_mask_detect<<<grid, 256, 0, s>>>(g, fa);
}

void launch_mask_count(const DevGraph &g, const FusedArgs &fa, hipStream_t s) {
    if (g.n_slots <= 0) return;
    k_mask_count<<<(g.n_slots + SWEEP_ROWS - 1) / SWEEP_ROWS, SWEEP_THREADS, 0, s>>>(g, fa);
}

void launch_edge_sweep(const DevGraph &g, const FusedArgs &fa, int32_t w, hipStream_t s) {
    if (g.n_slots <= 0) return;
    k_edge_sweep<<<(g.n_slots + SWEEP_ROWS - 1) / SWEEP_ROWS, SWEEP_THREADS, 0, s>>>(g, fa, w);
}

void launch_count_flag_rows(const DevGraph &g, const FusedArgs &fa, hipStream_t s) {
    k_count_flag_rows<<<1, 256, 0, s>>>(g, fa);
}

int32_t launch_mask_recompute(const DevGraph &g, const FusedArgs &fa, int32_t reset_only, hipStream_t s) {
    if (g.n_slots <= 0) return 0;
    const int blocks = std::min(RECOMPUTE_BLOCKS, (g.n_slots + RECOMPUTE_WAVES - 1) / RECOMPUTE_WAVES);
    k_recompute_rows<<<blocks, 64 * RECOMPUTE_WAVES, 0, s>>>(g, fa, reset_only);
    if (reset_only) return -blocks;  // no heavy-row pass: its partials are not summed
    k_fused_heavy<<<FUSED_GRID, FUSED_THREADS, fused_lds_bytes(g.P), s>>>(g, fa);
    return blocks;
}

static_assert(APSP_MAX_CAPACITY % TILE == 0, "capacity limit must be a tile multiple");
static_assert(((size_t)APSP_MAX_CAPACITY + 2 * (APSP_MAX_CAPACITY / 32) + LDS_LIST + 64) * 4 <= 163840,
              "a row of the largest graph must fit in LDS");

hipError_t configure_kernels() {
    static hipError_t status = hipErrorNotReady;
    if (status != hipErrorNotReady) return status;
    status = hipFuncSetAttribute((const void *)k_fused_heavy, hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)fused_lds_bytes(APSP_MAX_CAPACITY));
    const int sel = (int)(nin_build_lds_bytes(APSP_MAX_CAPACITY) + sizeof(SelectShared));
    if (status == hipSuccess)
        status = hipFuncSetAttribute((const void *)k_nin_build, hipFuncAttributeMaxDynamicSharedMemorySize, sel);
    if (status == hipSuccess)
        status = hipFuncSetAttribute((const void *)k_select_vec, hipFuncAttributeMaxDynamicSharedMemorySize, sel);
    if (status == hipSuccess)
        status = hipFuncSetAttribute((const void *)k_nin_rebuild_queue, hipFuncAttributeMaxDynamicSharedMemorySize, sel);
    if (status == hipSuccess)
        status = hipFuncSetAttribute((const void *)k_edge_begin, hipFuncAttributeMaxDynamicSharedMemorySize, sel);
    (void)hipGetLastError();  // do not leave the status for an unrelated launch check
    return status;
}

APSP_SR_END
}  // namespace apsp
