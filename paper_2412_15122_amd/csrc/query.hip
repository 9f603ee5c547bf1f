// Warm single-pair queries: the path (Section 4, Algorithm 7; for minimax
// graphs a search over edges no heavier than the distance), the nodes on
// some / on every shortest path (Algorithms 8 and 10), matrix read-out, and
// the edge scope count.
#include <vector>

#include "device_common.h"

namespace apsp {
APSP_SR_BEGIN

__global__ __launch_bounds__(1024) void k_query(DevGraph g, int32_t si, int32_t sj, int32_t *out,
                                                int32_t *scratch) {
    query_block(g, si, sj, out, scratch);
}

void launch_query(const DevGraph &g, int32_t si, int32_t sj, int32_t *out, int32_t *scratch, hipStream_t s) {
    k_query<<<1, 1024, 0, s>>>(g, si, sj, out, scratch);
}

// Algorithm 8's paths through the candidates cand[0..count): work-group c
// writes the path si -> cand[c] and then cand[c] -> sj, each as query_block
// does (3 + P words from out + 2 c (P + 3)), over its own 4 P words of
// scratch.
__global__ __launch_bounds__(1024) void k_query_paths(DevGraph g, int32_t si, int32_t sj, const int32_t *cand,
                                                      int32_t *out, int32_t *scratch) {
    const int32_t c = blockIdx.x;
    const int32_t t = cand[c];
    int32_t *sc = scratch + (int64_t)c * 4 * g.P;
    int32_t *o = out + (int64_t)c * 2 * (g.P + 3);
    query_block(g, si, t, o, sc);
    __syncthreads();
    query_block(g, t, sj, o + g.P + 3, sc);
}

void launch_query_paths(const DevGraph &g, int32_t si, int32_t sj, const int32_t *cand, int32_t count, int32_t *out,
                        int32_t *scratch, hipStream_t s) {
    if (count > 0) k_query_paths<<<count, 1024, 0, s>>>(g, si, sj, cand, out, scratch);
}

#ifdef APSP_SEMIRING_MINIMAX
// ---- a minimax path of a pair ------------------------------------------------
// With max in place of +, Algorithm 7's candidate set keeps most of the graph
// (ties are the rule: on an undirected graph minimax distances form an
// ultrametric), so the path is found directly: every walk from i to j over
// edges of weight <= d = D[i][j] is a minimax path, and a breadth-first
// search from i over those edges, one launch per level, reaches j.  Its
// parent tree gives a simple path (fewest edges among them).
// Scratch (4 P ints): parent[P], two frontiers of P, the visited bitmap
// (P / 32 words), then QB_CTL control words.
constexpr int QB_LEVELS_PER_SYNC = 16;
constexpr int QB_GRID = 1024;
enum QbCtl { QB_COUNT0 = 0, QB_COUNT1, QB_COUNT2, QB_FOUND, QB_EMPTY, QB_CTL };

struct QbView {
    int32_t *parent, *f0, *f1;
    uint32_t *visited;
    int32_t *ctl;
};

__host__ __device__ inline QbView qb_view(int32_t *scratch, int32_t P) {
    QbView v;
    v.parent = scratch;
    v.f0 = scratch + P;
    v.f1 = scratch + 2 * P;
    v.visited = (uint32_t *)(scratch + 3 * P);
    v.ctl = scratch + 3 * P + (P + 31) / 32;
    return v;
}

__global__ __launch_bounds__(256) void k_qb_init(DevGraph g, int32_t si, int32_t sj, int32_t *scratch) {
    const QbView v = qb_view(scratch, g.P);
    const int32_t w = blockIdx.x * blockDim.x + threadIdx.x;
    if (w < (g.P + 31) / 32) v.visited[w] = w == (si >> 5) ? 1u << (si & 31) : 0u;
    if (w == 0) {
        v.ctl[QB_COUNT0] = 1;
        v.ctl[QB_COUNT1] = 0;
        v.ctl[QB_COUNT2] = 0;
        v.ctl[QB_FOUND] = si == sj;
        v.ctl[QB_EMPTY] = 0;
        v.f0[0] = si;
        v.parent[si] = -1;
    }
}

// Level `level`: every edge a -> b of weight <= d out of the level's frontier
// to an unvisited b puts b on the next frontier.  One wavefront per (frontier
// node, 1024-column chunk) work item, grid-stride.  Frontier sizes rotate
// through three counters: level l reads count l % 3, adds to (l + 1) % 3 and
// zeroes (l + 2) % 3 for the level after.  Once j is reached, or a frontier
// is empty (also when j is unreachable), a sticky flag ends every later level.
__global__ __launch_bounds__(256) void k_qb_level(DevGraph g, int32_t si, int32_t sj, int32_t skip, int32_t level,
                                                  int32_t *scratch) {
    const QbView v = qb_view(scratch, g.P);
    if (v.ctl[QB_FOUND] || v.ctl[QB_EMPTY]) return;
    const uint32_t d = (uint32_t)g.D[(int64_t)si * g.ld + sj];
    const int32_t cnt_in = v.ctl[QB_COUNT0 + level % 3];
    if (cnt_in == 0 || d >= INF) {
        if (threadIdx.x == 0) v.ctl[QB_EMPTY] = 1;
        return;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) v.ctl[QB_COUNT0 + (level + 2) % 3] = 0;  // the level after next
    int32_t *cnt_out = &v.ctl[QB_COUNT0 + (level + 1) % 3];
    const int32_t *fin = level % 2 ? v.f1 : v.f0;
    int32_t *fout = level % 2 ? v.f0 : v.f1;
    const int n = g.n_slots;
    const int32_t chunks = (n + 1023) / 1024;
    const int64_t items = (int64_t)cnt_in * chunks;
    const int lane = lane_id();
    for (int64_t it = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); it < items; it += (int64_t)gridDim.x * 4) {
        const int32_t a = fin[it / chunks];
        const int32_t cb = (int32_t)(it % chunks) * 1024;
        const int32_t *arow = g.A + (int64_t)a * g.ld;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int32_t b0 = cb + q * 256 + lane * 4;
            uint32_t take = 0;
            if (b0 < n) {
                const uint4 wv = *reinterpret_cast<const uint4 *>(arow + b0);
                const uint32_t ws[4] = {wv.x, wv.y, wv.z, wv.w};
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int32_t b = b0 + e;
                    if (b >= n || b == a || b == skip || ws[e] > d) continue;
                    const uint32_t bit = 1u << (b & 31);
                    if (v.visited[b >> 5] & bit) continue;
                    if (atomicOr(&v.visited[b >> 5], bit) & bit) continue;
                    v.parent[b] = a;
                    take |= 1u << e;
                    if (b == sj) atomicExch(&v.ctl[QB_FOUND], 1);
                }
            }
            // one counter atomic per wavefront for the nodes it took
            const int mine = __popc(take);
            int incl = mine;
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
                const int t = __shfl_up(incl, o);
                if (lane >= o) incl += t;
            }
            const int total = __shfl(incl, 63);
            int base = 0;
            if (lane == 63 && total) base = atomicAdd(cnt_out, total);
            base = __shfl(base, 63);
            int pos = base + incl - mine;
            for (int e = 0; e < 4; ++e)
                if (take >> e & 1u) fout[pos++] = b0 + e;
        }
    }
}

// The path from the parent tree: out = dist, length, error, ids from i to j.
__global__ void k_qb_path(DevGraph g, int32_t si, int32_t sj, int32_t *out, const int32_t *scratch) {
    const QbView v = qb_view(const_cast<int32_t *>(scratch), g.P);
    const uint32_t d = (uint32_t)g.D[(int64_t)si * g.ld + sj];
    if (si == sj) { out[0] = 0; out[1] = 1; out[2] = 0; out[3] = g.id_of_slot[si]; return; }
    if (d >= INF) { out[0] = (int32_t)INF; out[1] = 0; out[2] = 0; return; }
    if (!v.ctl[QB_FOUND]) { out[0] = (int32_t)d; out[1] = 0; out[2] = 1; return; }
    int32_t len = 1;
    int32_t c0 = sj;
    for (; c0 >= 0 && c0 != si && len <= g.n_slots; c0 = v.parent[c0]) ++len;
    if (c0 != si) { out[0] = (int32_t)d; out[1] = 0; out[2] = 1; return; }
    int32_t c = sj;
    for (int32_t p = len - 1; p >= 0; --p) {
        out[3 + p] = g.id_of_slot[c];
        c = v.parent[c];
    }
    out[0] = (int32_t)d;
    out[1] = len;
    out[2] = 0;
}

// The search from si, not entering slot `skip` (-1: none); on return the
// probe holds the control words (QB_FOUND: sj reached).
static const char *qb_search(const DevGraph &g, int32_t si, int32_t sj, int32_t skip, int32_t *scratch,
                             int32_t *probe_host, hipStream_t s) {
    k_qb_init<<<((g.P + 31) / 32 + 255) / 256, 256, 0, s>>>(g, si, sj, scratch);
    const QbView v = qb_view(scratch, g.P);
    probe_host[QB_FOUND] = si == sj;
    for (int32_t level = 0; si != sj && level < g.n_slots; level += QB_LEVELS_PER_SYNC) {
        for (int32_t l = level; l < level + QB_LEVELS_PER_SYNC; ++l)
            k_qb_level<<<QB_GRID, 256, 0, s>>>(g, si, sj, skip, l, scratch);
        if (hipMemcpyAsync(probe_host, v.ctl, QB_CTL * 4, hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return "query level sync";
        if (probe_host[QB_FOUND] || probe_host[QB_EMPTY]) break;
    }
    return nullptr;
}

const char *launch_query_bottleneck(const DevGraph &g, int32_t si, int32_t sj, int32_t *out, int32_t *scratch,
                                    int32_t *probe_host, hipStream_t s) {
    if (const char *bad = qb_search(g, si, sj, -1, scratch, probe_host, s)) return bad;
    k_qb_path<<<1, 1, 0, s>>>(g, si, sj, out, scratch);
    return nullptr;
}

// The slots of the found path, sj first: path[0] = length, path[1..] slots
// (length 0 when sj was not reached).
__global__ void k_qb_path_slots(DevGraph g, int32_t si, int32_t sj, int32_t *path, const int32_t *scratch) {
    const QbView v = qb_view(const_cast<int32_t *>(scratch), g.P);
    int32_t len = 0;
    if (v.ctl[QB_FOUND]) {
        int32_t c = sj;
        for (; c >= 0 && len < g.n_slots; c = c == si ? -1 : v.parent[c]) path[1 + len++] = c;
        if (path[len] != si) len = 0;
    }
    path[0] = len;
}

__global__ void k_qb_mark(int32_t *mark, int32_t slot) { mark[slot] = 1; }

// The ids of the marked slots in ascending-id order (rank table), at
// out[4 + n_live ...], their count at out[2].
__global__ __launch_bounds__(1024) void k_qb_emit_marked(DevGraph g, const int32_t *__restrict__ rank, int32_t n_live,
                                                         const int32_t *mark, int32_t *out) {
    __shared__ uint32_t red[16];
    __shared__ int s_base;
    if (threadIdx.x == 0) s_base = 0;
    __syncthreads();
    for (int32_t r0 = 0; r0 < n_live; r0 += 1024) {
        const int32_t r = r0 + threadIdx.x;
        const int32_t slot = r < n_live ? rank[r] : -1;
        const int key = slot >= 0 && mark[slot];
        int total;
        const int off = block_exscan<1024>(key, red, &total);
        if (key) out[4 + n_live + s_base + off] = g.id_of_slot[slot];
        __syncthreads();
        if (threadIdx.x == 0) s_base += total;
        __syncthreads();
    }
    if (threadIdx.x == 0) out[2] = s_base;
}

#endif

// ---- nodes on some / on every shortest path of a pair ----------------------
// (Algorithms 7 and 8 give the candidates and the paths through them,
// Theorem 5; Algorithm 10 intersects the pair's shortest paths.)
//
// Levels: L[t] = D[i][t].  Along a tight edge x -> y (both candidates,
// L[x] + A[x][y] == L[y]) the level does not fall, and the tight walks from
// i to j are exactly the shortest i -> j walks.  A candidate t other than i
// and j is on every such walk iff (a) no tight edge jumps over its level
// (L[x] < L[t] < L[y]) and (b) no walk crosses level L[t] avoiding t: with no
// zero-weight tight edge inside the level, (b) holds iff t is alone on it;
// otherwise a search inside the level decides, from the nodes entered from
// below (or i) to the nodes that leave upward (or j).
//
// Scratch (4 P ints): cand[K] slots in ascending-id order, lev[K], reach[K]
// (highest level a tight out-edge reaches, -1 if none), flags[K].
// Output (4 + 2 n_live ints): dist, K, number of key nodes, 0, the K
// candidate ids, then (at 4 + n_live) the key ids, both ascending.
constexpr int QN_ENTRY = 1;  // a tight in-edge from a lower level
constexpr int QN_INTRA = 2;  // a zero-weight tight edge to or from the same level
constexpr int QN_KEY = 4;
constexpr int QN_GRID = 256;  // work-groups of the per-candidate pass
// The caller places the output (2 P + 8 ints, rounded up) and QN_GRID search
// spaces of 2 P ints in the heavy-pass scratch of FUSED_GRID * 2 P ints.
static_assert(2 * QN_GRID + 3 <= 2 * FUSED_GRID, "query-nodes scratch exceeds the heavy-pass scratch");

__global__ __launch_bounds__(1024) void k_qn_gather(DevGraph g, int32_t si, int32_t sj, const int32_t *__restrict__ rank,
                                                    int32_t n_live, int32_t *out, int32_t *scratch) {
    __shared__ uint32_t red[16];
    __shared__ int s_base;
    int32_t *cand = scratch, *lev = scratch + g.P, *reach = scratch + 2 * g.P, *flags = scratch + 3 * g.P;
    const int64_t ld = g.ld;
    const uint32_t dist = (uint32_t)g.D[(int64_t)si * ld + sj];
    if (threadIdx.x == 0) s_base = 0;
    __syncthreads();
    for (int32_t r0 = 0; r0 < n_live; r0 += 1024) {
        const int32_t r = r0 + threadIdx.x;
        int32_t t = -1;
        uint32_t lt = 0;
        if (r < n_live && dist < INF) {
            t = rank[r];
            lt = (uint32_t)g.D[(int64_t)si * ld + t];
            const uint32_t tj = (uint32_t)g.D[(int64_t)t * ld + sj];
            const bool on = si == sj ? t == si : cat(lt, tj) == dist;
            if (!on) t = -1;
        }
        int total;
        const int off = block_exscan<1024>(t >= 0, red, &total);
        const int c = s_base + off;
        if (t >= 0) {
            cand[c] = t;
            lev[c] = (int32_t)lt;
            reach[c] = -1;
            flags[c] = 0;
            out[4 + c] = g.id_of_slot[t];
        }
        __syncthreads();
        if (threadIdx.x == 0) s_base += total;
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = (int32_t)dist;
        out[1] = s_base;
        out[2] = 0;
        out[3] = 0;
    }
}

// One wave per candidate x: its tight out-edges to other candidates.
__global__ __launch_bounds__(256) void k_qn_edges(DevGraph g, const int32_t *out, int32_t *scratch) {
    const int32_t K = out[1];
    const int32_t x = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (x >= K) return;
    int32_t *cand = scratch, *lev = scratch + g.P, *reach = scratch + 2 * g.P, *flags = scratch + 3 * g.P;
    const int32_t *arow = g.A + (int64_t)cand[x] * g.ld;
    const uint32_t lx = (uint32_t)lev[x];
    int32_t hi = -1;
    int intra = 0;
    for (int32_t y = lane_id(); y < K; y += 64) {
        const uint32_t a = (uint32_t)arow[cand[y]];
        const uint32_t ly = (uint32_t)lev[y];
        if (y == x || a >= INF || cat(lx, a) != ly) continue;
        if (ly > lx) {
            hi = max(hi, (int32_t)ly);
            atomicOr(&flags[y], QN_ENTRY);
        } else {
            intra = 1;
            atomicOr(&flags[y], QN_INTRA);
        }
    }
    hi = (int32_t)wave_max((uint32_t)(hi + 1)) - 1;
    intra = __any(intra);
    if (lane_id() == 0) {
        reach[x] = hi;
        if (intra) atomicOr(&flags[x], QN_INTRA);
    }
}

// Is candidate t on every tight i -> j walk?  One work-group per candidate
// (grid-stride); `bfs` holds 2 P ints per work-group.
__global__ __launch_bounds__(256) void k_qn_key(DevGraph g, int32_t si, int32_t sj, const int32_t *out,
                                                int32_t *scratch, int32_t *bfs) {
    __shared__ uint32_t vis[APSP_MAX_CAPACITY / 32 + 1];
    __shared__ int s_m, s_tail, s_found;
    const int32_t K = out[1];
    int32_t *cand = scratch, *lev = scratch + g.P, *reach = scratch + 2 * g.P, *flags = scratch + 3 * g.P;
    int32_t *mem = bfs + (int64_t)blockIdx.x * 2 * g.P;  // level members (candidate indices)
    int32_t *q = mem + g.P;                              // search queue (member indices)
    const int tid = threadIdx.x;
    for (int32_t t = blockIdx.x; t < K; t += gridDim.x) {
        const int32_t st = cand[t];
        if (st == si || st == sj) continue;
        const int32_t lt = lev[t];
        int jumped = 0, same = 0, intra = 0;
        for (int32_t x = tid; x < K; x += 256) {
            const int32_t lx = lev[x];
            jumped |= lx < lt && reach[x] > lt;
            same |= x != t && lx == lt;
            intra |= lx == lt && (flags[x] & QN_INTRA);
        }
        jumped = __syncthreads_or(jumped);
        same = __syncthreads_or(same);
        intra = __syncthreads_or(intra);
        bool key;
        if (jumped) {
            key = false;
        } else if (!same) {
            key = true;
        } else if (!intra) {
            key = false;
        } else {
            // Search inside level lt, without t, from the entries to the exits.
            if (tid == 0) { s_m = 0; s_tail = 0; s_found = 0; }
            __syncthreads();
            for (int32_t x = tid; x < K; x += 256)
                if (x != t && lev[x] == lt) mem[atomicAdd(&s_m, 1)] = x;
            __syncthreads();
            const int M = s_m;
            for (int w = tid; w < (M + 31) / 32; w += 256) vis[w] = 0;
            __syncthreads();
            for (int m = tid; m < M; m += 256) {
                const int32_t x = mem[m];
                if (cand[x] == si || (flags[x] & QN_ENTRY)) {
                    atomicOr(&vis[m >> 5], 1u << (m & 31));
                    q[atomicAdd(&s_tail, 1)] = m;
                    if (cand[x] == sj || reach[x] > lt) s_found = 1;
                }
            }
            __syncthreads();
            int head = 0, tail = s_tail;
            __syncthreads();
            while (!s_found && head < tail) {
                const int64_t pairs = (int64_t)(tail - head) * M;
                for (int64_t e = tid; e < pairs; e += 256) {
                    const int a = q[head + (int)(e / M)], b = (int)(e % M);
                    if ((vis[b >> 5] >> (b & 31)) & 1u) continue;
                    if (g.A[(int64_t)cand[mem[a]] * g.ld + cand[mem[b]]] != 0) continue;
                    const uint32_t was = atomicOr(&vis[b >> 5], 1u << (b & 31));
                    if ((was >> (b & 31)) & 1u) continue;
                    q[atomicAdd(&s_tail, 1)] = b;
                    const int32_t y = mem[b];
                    if (cand[y] == sj || reach[y] > lt) s_found = 1;
                }
                __syncthreads();
                head = tail;
                tail = s_tail;
                __syncthreads();
            }
            key = !s_found;
            __syncthreads();
        }
        if (key && tid == 0) atomicOr(&flags[t], QN_KEY);
    }
}

// The key ids, ascending (candidates are in ascending-id order).
__global__ __launch_bounds__(1024) void k_qn_emit(DevGraph g, int32_t n_live, int32_t *out, const int32_t *scratch) {
    __shared__ uint32_t red[16];
    __shared__ int s_base;
    const int32_t K = out[1];
    const int32_t *cand = scratch, *flags = scratch + 3 * g.P;
    if (threadIdx.x == 0) s_base = 0;
    __syncthreads();
    for (int32_t c0 = 0; c0 < K; c0 += 1024) {
        const int32_t c = c0 + threadIdx.x;
        const int key = c < K && (flags[c] & QN_KEY);
        int total;
        const int off = block_exscan<1024>(key, red, &total);
        if (key) out[4 + n_live + s_base + off] = g.id_of_slot[cand[c]];
        __syncthreads();
        if (threadIdx.x == 0) s_base += total;
        __syncthreads();
    }
    if (threadIdx.x == 0) out[2] = s_base;
}

void launch_query_nodes(const DevGraph &g, int32_t si, int32_t sj, const int32_t *rank, int32_t n_live,
                        int32_t *out, int32_t *scratch, int32_t *bfs, hipStream_t s) {
    k_qn_gather<<<1, 1024, 0, s>>>(g, si, sj, rank, n_live, out, scratch);
    k_qn_edges<<<(n_live + 3) / 4, 256, 0, s>>>(g, out, scratch);
    k_qn_key<<<QN_GRID, 256, 0, s>>>(g, si, sj, out, scratch, bfs);
    k_qn_emit<<<1, 1024, 0, s>>>(g, n_live, out, scratch);
}

#ifdef APSP_SEMIRING_MINIMAX
// Node sets of a minimax pair.  The set on optimal walks is the gather of
// k_qn_gather (max in place of +); the nodes on every optimal walk all lie
// on the one path the search finds, and such a node t is one of them when
// the search without t does not reach sj.  work: 5 P + 64 ints (the
// gather's candidate arrays, the path, the marks).
const char *launch_query_nodes_bottleneck(const DevGraph &g, int32_t si, int32_t sj, const int32_t *rank,
                                          int32_t n_live, int32_t *out, int32_t *scratch, int32_t *work,
                                          int32_t *probe_host, hipStream_t s) {
    int32_t *cand = work;                  // 4 P: the gather's candidate arrays
    int32_t *path = work + 4 * g.P;        // P + 1
    int32_t *mark = out + 4 + 2 * (int64_t)n_live;  // n_slots marks after the output lists
    k_qn_gather<<<1, 1024, 0, s>>>(g, si, sj, rank, n_live, out, cand);
    launch_fill(mark, g.n_slots, 0, s);
    if (si != sj) {
        if (const char *bad = qb_search(g, si, sj, -1, scratch, probe_host, s)) return bad;
        k_qb_path_slots<<<1, 1, 0, s>>>(g, si, sj, path, scratch);
        if (hipMemcpyAsync(probe_host, path, 4, hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return "query path length";
        const int32_t len = probe_host[0];
        std::vector<int32_t> slots(len > 0 ? len : 0);
        if (len > 0 && (hipMemcpyAsync(slots.data(), path + 1, (size_t)len * 4, hipMemcpyDeviceToHost, s) != hipSuccess ||
                        hipStreamSynchronize(s) != hipSuccess))
            return "query path";
        for (int32_t q = 1; q + 1 < len; ++q) {  // interior nodes of the path
            if (const char *bad = qb_search(g, si, sj, slots[q], scratch, probe_host, s)) return bad;
            if (!probe_host[QB_FOUND]) k_qb_mark<<<1, 1, 0, s>>>(mark, slots[q]);
        }
    }
    k_qb_emit_marked<<<1, 1024, 0, s>>>(g, rank, n_live, mark, out);
    return nullptr;
}
#endif

// dst[a][b] = src[slot[a]][slot[b]] for a, b < n.
__global__ void k_gather_compact(const int32_t *__restrict__ src, int64_t ld, int32_t *__restrict__ dst,
                                 int64_t dst_ld, const int32_t *__restrict__ slot, int32_t n, int32_t widest) {
    const int32_t b = blockIdx.x * blockDim.x + threadIdx.x;
    const int32_t a = blockIdx.y;
    if (b >= n) return;
    const int32_t v = src[(int64_t)slot[a] * ld + slot[b]];
    dst[(int64_t)a * dst_ld + b] = widest ? widest_xf(v) : v;
}

void launch_gather_compact(const int32_t *src, int64_t ld, int32_t *dst, int64_t dst_ld,
                           const int32_t *slot_of_rank, int32_t n, int32_t widest, hipStream_t s) {
    if (n <= 0) return;
    dim3 grid((n + 255) / 256, n);
    k_gather_compact<<<grid, 256, 0, s>>>(src, ld, dst, dst_ld, slot_of_rank, n, widest);
}

// |R| and |C| of edge su -> sv at its current weight.
__global__ void k_edge_scope(DevGraph g, int32_t su, int32_t sv) {
    __shared__ int red_r[4], red_c[4];
    const int32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t ld = g.ld;
    const uint32_t w = (uint32_t)g.A[(int64_t)su * ld + sv];
    int r = 0, c = 0;
    if (t < g.n_slots && g.id_of_slot[t] >= 0) {
        const uint32_t du = (uint32_t)g.D[(int64_t)t * ld + su], dv = (uint32_t)g.D[(int64_t)t * ld + sv];
        r = (dv < INF && cat(du, w) == dv);
        const uint32_t ru = (uint32_t)g.D[(int64_t)su * ld + t], rv = (uint32_t)g.D[(int64_t)sv * ld + t];
        c = (ru < INF && cat(w, rv) == ru);
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        r += __shfl_xor(r, o);
        c += __shfl_xor(c, o);
    }
    if ((threadIdx.x & 63) == 0) {
        red_r[threadIdx.x >> 6] = r;
        red_c[threadIdx.x >> 6] = c;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        atomicAdd(&g.ctl->scope_r, red_r[0] + red_r[1] + red_r[2] + red_r[3]);
        atomicAdd(&g.ctl->scope_c, red_c[0] + red_c[1] + red_c[2] + red_c[3]);
    }
}

void launch_edge_scope(const DevGraph &g, int32_t su, int32_t sv, hipStream_t s) {
    if (g.n_slots <= 0) return;
    k_edge_scope<<<(g.n_slots + 255) / 256, 256, 0, s>>>(g, su, sv);
}

APSP_SR_END
}  // namespace apsp
