// Warm single-pair query (Section 3, Algorithm 7), matrix read-out, and the
// edge scope count.
#include "device_common.h"

namespace apsp {

__global__ __launch_bounds__(1024) void k_query(DevGraph g, int32_t si, int32_t sj, int32_t *out,
                                                int32_t *scratch) {
    query_block(g, si, sj, out, scratch);
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
