// Warm single-pair query (Section 3, Algorithm 7), matrix read-out, and the
// edge scope count.
#include "apsp_internal.h"

namespace apsp {

__device__ __forceinline__ uint32_t q_wave_min(uint32_t v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = min(v, (uint32_t)__shfl_xor((int)v, o));
    return v;
}

// Block-wide minimum of a 64-bit key for 1024 threads.
__device__ unsigned long long block_min_key(unsigned long long v, unsigned long long *red) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)v, o);
        uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)(v >> 32), o);
        unsigned long long w = ((unsigned long long)hi << 32) | lo;
        v = w < v ? w : v;
    }
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    unsigned long long r = red[0];
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w) r = red[w] < r ? red[w] : r;
    return r;
}

// out[0] = dist, out[1] = path length, out[2] = status (0 ok, 1 no path
// found), out[3..] = path ids.  scratch holds 4 * P ints.
//
// Candidates (Algorithm 7): t with D[i][t] + D[t][j] == D[i][j], plus i
// and j; by Theorem al_correct they contain every shortest i -> j path.
// The walk takes, from cur, the candidate b with the smallest id such that
// A[cur][b] + D[b][j] == D[cur][j] (the edge starts a shortest path to j).
// With weights >= 1 this yields the lexicographically smallest shortest
// path.  Zero-weight edges can trap the greedy walk in a zero cycle; then a
// breadth-first search over the same tight edges returns a shortest simple
// path instead.
__global__ __launch_bounds__(1024) void k_query(DevGraph g, int32_t si, int32_t sj, int32_t *out,
                                                int32_t *scratch) {
    __shared__ unsigned long long red[16];
    __shared__ int32_t s_k, s_ci, s_cj, s_changed;
    __shared__ uint32_t visited[APSP_MAX_CAPACITY / 32 + 32];
    const int tid = threadIdx.x;
    const int n = g.n_slots;
    const int64_t ld = g.ld;
    int32_t *cand = scratch;
    int32_t *candD = scratch + g.P;
    int32_t *lvl = scratch + 2 * g.P;
    int32_t *parent = scratch + 3 * g.P;
    const uint32_t dist = (uint32_t)g.D[(int64_t)si * ld + sj];
    if (si == sj) {
        if (tid == 0) { out[0] = 0; out[1] = 1; out[2] = 0; out[3] = g.id_of_slot[si]; }
        return;
    }
    if (dist >= INF) {
        if (tid == 0) { out[0] = (int32_t)INF; out[1] = 0; out[2] = 0; }
        return;
    }
    if (tid == 0) { s_k = 0; s_ci = -1; s_cj = -1; }
    for (int w = tid; w < (n + 31) / 32; w += blockDim.x) visited[w] = 0;
    __syncthreads();
    for (int32_t t = tid; t < n; t += blockDim.x) {
        if (g.id_of_slot[t] < 0) continue;
        const uint32_t dit = (uint32_t)g.D[(int64_t)si * ld + t];
        const uint32_t dtj = (uint32_t)g.D[(int64_t)t * ld + sj];
        if (t == si || t == sj || dit + dtj == dist) {
            const int c = atomicAdd(&s_k, 1);
            cand[c] = t;
            candD[c] = (int32_t)dtj;
            if (t == si) s_ci = c;
            if (t == sj) s_cj = c;
        }
    }
    __syncthreads();
    const int K = s_k;
    // greedy walk
    int32_t cur = si;
    uint32_t dcur = dist;
    int len = 0;
    if (tid == 0) out[3] = g.id_of_slot[si];
    len = 1;
    if (tid == 0) atomicOr(&visited[si >> 5], 1u << (si & 31));
    bool stuck = false;
    while (cur != sj) {
        __syncthreads();
        unsigned long long best = ~0ull;
        for (int c = tid; c < K; c += blockDim.x) {
            const int32_t b = cand[c];
            if (b == cur || (visited[b >> 5] >> (b & 31)) & 1u) continue;
            const uint32_t a = (uint32_t)g.A[(int64_t)cur * ld + b];
            if (a >= INF) continue;
            if (a + (uint32_t)candD[c] == dcur) {
                const unsigned long long key = ((unsigned long long)(uint32_t)g.id_of_slot[b] << 32) | (uint32_t)c;
                best = key < best ? key : best;
            }
        }
        best = block_min_key(best, red);
        if (best == ~0ull || len >= K) {
            stuck = true;
            break;
        }
        const int c = (int)(uint32_t)best;
        cur = cand[c];
        dcur = (uint32_t)candD[c];
        if (tid == 0) {
            out[3 + len] = (int32_t)(best >> 32);
            atomicOr(&visited[cur >> 5], 1u << (cur & 31));
        }
        ++len;
    }
    if (!stuck) {
        if (tid == 0) { out[0] = (int32_t)dist; out[1] = len; out[2] = 0; }
        return;
    }
    // breadth-first search over tight edges a -> b (A[a][b] + D[b][j] == D[a][j])
    const int ci = s_ci, cj = s_cj;
    for (int c = tid; c < K; c += blockDim.x) { lvl[c] = -1; parent[c] = -1; }
    __syncthreads();
    if (tid == 0) lvl[ci] = 0;
    int level = 0;
    for (;;) {
        __syncthreads();
        if (tid == 0) s_changed = 0;
        __syncthreads();
        for (int c2 = tid; c2 < K; c2 += blockDim.x) {
            if (lvl[c2] != -1) continue;
            const int32_t b = cand[c2];
            for (int c = 0; c < K; ++c) {
                if (lvl[c] != level) continue;
                const int32_t a = cand[c];
                if (a == b) continue;
                const uint32_t w = (uint32_t)g.A[(int64_t)a * ld + b];
                if (w < INF && w + (uint32_t)candD[c2] == (uint32_t)candD[c]) {
                    lvl[c2] = level + 1;
                    parent[c2] = c;
                    s_changed = 1;
                    break;
                }
            }
        }
        __syncthreads();
        if (lvl[cj] != -1 || s_changed == 0) break;
        ++level;
    }
    if (tid == 0) {
        if (lvl[cj] == -1) {
            out[0] = (int32_t)dist; out[1] = 0; out[2] = 1;
        } else {
            const int L = lvl[cj] + 1;
            int c = cj;
            for (int p = L - 1; p >= 0; --p) {
                out[3 + p] = g.id_of_slot[cand[c]];
                c = parent[c];
            }
            out[0] = (int32_t)dist; out[1] = L; out[2] = 0;
        }
    }
}

void launch_query(const DevGraph &g, int32_t si, int32_t sj, int32_t *out, int32_t *scratch, hipStream_t s) {
    k_query<<<1, 1024, 0, s>>>(g, si, sj, out, scratch);
}

// dst[a][b] = src[slot[a]][slot[b]] for a, b < n.
__global__ void k_gather_compact(const int32_t *__restrict__ src, int64_t ld, int32_t *__restrict__ dst,
                                 int64_t dst_ld, const int32_t *__restrict__ slot, int32_t n) {
    const int32_t b = blockIdx.x * blockDim.x + threadIdx.x;
    const int32_t a = blockIdx.y;
    if (b >= n) return;
    dst[(int64_t)a * dst_ld + b] = src[(int64_t)slot[a] * ld + slot[b]];
}

void launch_gather_compact(const int32_t *src, int64_t ld, int32_t *dst, int64_t dst_ld,
                           const int32_t *slot_of_rank, int32_t n, hipStream_t s) {
    if (n <= 0) return;
    dim3 grid((n + 255) / 256, n);
    k_gather_compact<<<grid, 256, 0, s>>>(src, ld, dst, dst_ld, slot_of_rank, n);
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
        r = (dv < INF && du + w == dv);
        const uint32_t ru = (uint32_t)g.D[(int64_t)su * ld + t], rv = (uint32_t)g.D[(int64_t)sv * ld + t];
        c = (ru < INF && w + rv == ru);
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

}  // namespace apsp
