// Cold start: adjacency load, transpose, and blocked Floyd-Warshall.
//
// Floyd-Warshall (the paper's cold baseline, Section 1) computes, for every
// pivot k, D[i][j] = min(D[i][j], D[i][k] (+) D[k][j]), with (+) the unit's
// semiring concatenation (+ for shortest paths, max for minimax paths).
// Blocked by 128-wide rounds it becomes, per round r with pivot block
// P = D[r][r]:
//   phase 1  P := closure of P (sequential pivots inside one work-group);
//   phase 2  row panel    D[r][j] := min(D[r][j], P (x) D[r][j]),
//            column panel D[i][r] := min(D[i][r], D[i][r] (x) P),
//            where (x) is the (min, (+)) product -- once P is closed, no
//            pivot order is needed inside a panel;
//   phase 3  every other tile D[i][j] := min(D[i][j], D[i][r] (x) D[r][j]).
// Integer min-plus and min-max are exact and order-free, and INF + INF
// (2^31) fits in uint32, so every schedule gives the same bits as the
// textbook loop.  Neither is a multiply-accumulate, so the tiles run on the
// vector ALUs, not on the matrix cores.
#include "apsp_internal.h"

namespace apsp {
APSP_SR_BEGIN

// ---------------------------------------------------------------------------
// small utilities
// ---------------------------------------------------------------------------

__global__ void k_fill(int32_t *__restrict__ p, int64_t count, int32_t v) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < count; i += stride) p[i] = v;
}

void launch_fill(int32_t *p, int64_t count, int32_t v, hipStream_t s) {
    if (count <= 0) return;
    int64_t blocks = (count + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    k_fill<<<(unsigned)blocks, 256, 0, s>>>(p, count, v);
}

__global__ void k_iota(int32_t *p, int32_t n) {
    int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = i;
}

void launch_iota(int32_t *p, int32_t n, hipStream_t s) {
    if (n <= 0) return;
    k_iota<<<(n + 255) / 256, 256, 0, s>>>(p, n);
}

// A[i][j] := adj[i][j] for i, j < n; diagonal 0; entries outside [0, INF]
// become INF and set the sticky error.  Undirected: the smaller of the two
// directions (an asymmetric pair also sets the error).
__global__ void k_load_adj(DevGraph g, const int32_t *__restrict__ adj, int64_t adj_ld, int32_t n) {
    int32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    int32_t i = blockIdx.y;
    if (j >= n || i >= n) return;
    int32_t w = adj[(int64_t)i * adj_ld + j];
    int bad = 0;
    if (w < 0 || (uint32_t)w > INF) { w = (int32_t)INF; bad = 1; }
    if (g.undirected) {
        int32_t w2 = adj[(int64_t)j * adj_ld + i];
        if (w2 < 0 || (uint32_t)w2 > INF) { w2 = (int32_t)INF; bad = 1; }
        if (w2 != w) bad = 1;
        w = min(w, w2);
    }
    if (g.widest) w = widest_xf(w);
    if (i == j) { w = 0; bad = 0; }
    g.A[(int64_t)i * g.ld + j] = w;
    if (bad) atomicOr(&g.ctl->err, (int32_t)ERR_VALUE);
}

void launch_load_adj(const DevGraph &g, const int32_t *adj, int64_t adj_ld, int32_t n, hipStream_t s) {
    if (n <= 0) return;
    dim3 grid((n + 255) / 256, n);
    k_load_adj<<<grid, 256, 0, s>>>(g, adj, adj_ld, n);
}

// dst = src^T over [0, n)^2 through 32x32 LDS tiles.
__global__ __launch_bounds__(256) void k_transpose(const int32_t *__restrict__ src, int32_t *__restrict__ dst,
                                                   int64_t ld, int32_t n) {
    __shared__ int32_t t[32][33];
    int32_t bx = blockIdx.x * 32, by = blockIdx.y * 32;
    int32_t tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
    for (int r = ty; r < 32; r += 8) {
        int32_t i = by + r, j = bx + tx;
        if (i < n && j < n) t[r][tx] = src[(int64_t)i * ld + j];
    }
    __syncthreads();
    for (int r = ty; r < 32; r += 8) {
        int32_t i = bx + r, j = by + tx;  // dst[i][j] = src[j][i]
        if (i < n && j < n) dst[(int64_t)i * ld + j] = t[tx][r];
    }
}

void launch_transpose(const int32_t *src, int32_t *dst, int64_t ld, int32_t n, hipStream_t s) {
    if (n <= 0) return;
    dim3 grid((n + 31) / 32, (n + 31) / 32);
    k_transpose<<<grid, 256, 0, s>>>(src, dst, ld, n);
}

__global__ void k_copy_square(int32_t *__restrict__ dst, const int32_t *__restrict__ src, int64_t ld, int32_t n) {
    int32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    int32_t i = blockIdx.y;
    if (j < n) dst[(int64_t)i * ld + j] = src[(int64_t)i * ld + j];
}

void launch_copy_square(int32_t *dst, const int32_t *src, int64_t ld, int32_t n, hipStream_t s) {
    if (n <= 0) return;
    dim3 grid((n + 255) / 256, n);
    k_copy_square<<<grid, 256, 0, s>>>(dst, src, ld, n);
}

// Import of a known distance matrix: D[i][j] := src[i][j] for i, j < n,
// checked against what the distance matrix of the loaded adjacency must
// satisfy (Section 1): every entry in [0, INF], a zero diagonal, no entry
// above its edge's weight (the edge alone is a path), and symmetry for an
// undirected graph.  Each failing entry adds one to *bad (one atomic per
// wave); an entry outside [0, INF] is stored as INF.
__global__ __launch_bounds__(256) void k_import_d(DevGraph g, const int32_t *__restrict__ src, int64_t src_ld,
                                                  int32_t n, int32_t *bad) {
    const int32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    const int32_t i = blockIdx.y;
    int b = 0;
    if (j < n) {
        const int32_t raw = src[(int64_t)i * src_ld + j];
        int32_t w = raw;
        if (w < 0 || (uint32_t)w > INF) { w = (int32_t)INF; b = 1; }
        if (g.widest) w = widest_xf(w);  // the checks below hold for the stored form
        if (i == j && w != 0) b = 1;
        if ((uint32_t)w > (uint32_t)g.A[(int64_t)i * g.ld + j]) b = 1;
        if (g.undirected && src[(int64_t)j * src_ld + i] != raw) b = 1;
        g.D[(int64_t)i * g.ld + j] = w;
    }
    const unsigned long long m = __ballot(b);
    if ((threadIdx.x & 63) == 0 && m) atomicAdd(bad, (int32_t)__popcll(m));
}

void launch_import_d(const DevGraph &g, const int32_t *src, int64_t src_ld, int32_t n, int32_t *bad, hipStream_t s) {
    if (n <= 0) return;
    dim3 grid((n + 255) / 256, n);
    k_import_d<<<grid, 256, 0, s>>>(g, src, src_ld, n, bad);
}

// *bad += #{(i, j) in [0, n)^2 : a[i][j] != b[i][j]} (one atomic per wave).
__global__ __launch_bounds__(256) void k_count_diff(const int32_t *__restrict__ a, int64_t lda,
                                                    const int32_t *__restrict__ b, int64_t ldb, int32_t n,
                                                    int32_t *bad, int32_t widest) {
    const int32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    const int32_t i = blockIdx.y;
    int32_t bv = j < n ? b[(int64_t)i * ldb + j] : 0;
    if (widest) bv = widest_xf(bv);
    const int d = j < n && a[(int64_t)i * lda + j] != bv;
    const unsigned long long m = __ballot(d);
    if ((threadIdx.x & 63) == 0 && m) atomicAdd(bad, (int32_t)__popcll(m));
}

void launch_count_diff(const int32_t *a, int64_t lda, const int32_t *b, int64_t ldb, int32_t n, int32_t *bad,
                       int32_t widest, hipStream_t s) {
    if (n <= 0) return;
    dim3 grid((n + 255) / 256, n);
    k_count_diff<<<grid, 256, 0, s>>>(a, lda, b, ldb, n, bad, widest);
}

// ---------------------------------------------------------------------------
// phase 1: closure of the 128 x 128 pivot block
// ---------------------------------------------------------------------------
// Thread t keeps row (t & 127), columns 16 * (t >> 7) + c, c < 16, of the
// block in registers for all 128 pivots.  Pivot k needs D[i][k] of every row
// and D[k][j] of every column; at the end of pivot k - 1 the owners of
// column k and of row k publish those values (already updated by pivot
// k - 1) to a two-deep LDS buffer, so one barrier per pivot suffices: pivot
// k reads buffer k & 1 while the next values go to the other.  During pivot
// k neither row k nor column k changes (D[k][k] is 0, or INF for a dead
// slot), so the published values are the ones the textbook loop reads.

__global__ __launch_bounds__(1024) void k_fw_pivot(int32_t *__restrict__ D, int64_t ld, int32_t r) {
    __shared__ __align__(16) uint32_t rowbuf[2][TILE];  // rowbuf[k & 1][j] = D[k][j]
    __shared__ uint32_t colbuf[2][TILE];                // colbuf[k & 1][i] = D[i][k]
    const int tid = threadIdx.x;
    const int row = tid & (TILE - 1);
    const int c0 = (tid >> 7) * 16;
    int32_t *src = D + ((int64_t)r * TILE + row) * ld + (int64_t)r * TILE + c0;
    uint32_t own[16];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int4 v = *reinterpret_cast<const int4 *>(src + 4 * q);
        own[4 * q + 0] = (uint32_t)v.x;
        own[4 * q + 1] = (uint32_t)v.y;
        own[4 * q + 2] = (uint32_t)v.z;
        own[4 * q + 3] = (uint32_t)v.w;
    }
    if (c0 == 0) colbuf[0][row] = own[0];
    if (row == 0) {
#pragma unroll
        for (int q = 0; q < 4; ++q)
            *reinterpret_cast<uint4 *>(&rowbuf[0][c0 + 4 * q]) =
                make_uint4(own[4 * q], own[4 * q + 1], own[4 * q + 2], own[4 * q + 3]);
    }
    __syncthreads();
    for (int kb = 0; kb < TILE; kb += 16) {
#pragma unroll
        for (int kk = 0; kk < 16; ++kk) {
            const int k = kb + kk;
            const int p = kk & 1;  // == k & 1: kb is even
            const uint32_t dik = colbuf[p][row];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const uint4 rk = *reinterpret_cast<const uint4 *>(&rowbuf[p][c0 + 4 * q]);
                own[4 * q + 0] = min(own[4 * q + 0], cat(dik, rk.x));
                own[4 * q + 1] = min(own[4 * q + 1], cat(dik, rk.y));
                own[4 * q + 2] = min(own[4 * q + 2], cat(dik, rk.z));
                own[4 * q + 3] = min(own[4 * q + 3], cat(dik, rk.w));
            }
            if (k + 1 < TILE) {
                if (c0 == ((k + 1) & ~15)) colbuf[p ^ 1][row] = own[(kk + 1) & 15];
                if (row == k + 1) {
#pragma unroll
                    for (int q = 0; q < 4; ++q)
                        *reinterpret_cast<uint4 *>(&rowbuf[p ^ 1][c0 + 4 * q]) =
                            make_uint4(own[4 * q], own[4 * q + 1], own[4 * q + 2], own[4 * q + 3]);
                }
            }
            __syncthreads();
        }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q)
        *reinterpret_cast<int4 *>(src + 4 * q) =
            make_int4((int)own[4 * q], (int)own[4 * q + 1], (int)own[4 * q + 2], (int)own[4 * q + 3]);
}

// ---------------------------------------------------------------------------
// phases 2 and 3: C := min(C, A (x) B) on 128 x 128 tiles
// ---------------------------------------------------------------------------
// 256 threads, each owning an 8 x 8 micro-tile: rows {4ty..4ty+3,
// 64+4ty..64+4ty+3} and columns {4tx.., 64+4tx..}.  The k dimension (128) is
// streamed through LDS in chunks of KC, A stored transposed so that every
// operand read is one 16-byte LDS load.  Two k steps are folded into one
// min of three (v_min3_u32).  C is read before and written after the whole
// k loop, so C may alias A or B (phase 2).

constexpr int KC = 32;
constexpr int LDS_W = TILE + 4;

__device__ __forceinline__ uint32_t umin3(uint32_t a, uint32_t b, uint32_t c) {
    return min(a, min(b, c));
}

__device__ __forceinline__ void minplus_tile(const int32_t *__restrict__ At, const int32_t *__restrict__ Bt,
                                             int32_t *Ct, int64_t ld, uint32_t (*As)[LDS_W],
                                             uint32_t (*Bs)[LDS_W], bool close = false) {
    const int tid = threadIdx.x;
    const int ty = tid >> 4, tx = tid & 15;
    uint32_t acc[8][8];
#pragma unroll
    for (int m = 0; m < 8; ++m) {
        int row = (m < 4) ? (ty * 4 + m) : (64 + ty * 4 + (m - 4));
        const int32_t *cp = Ct + (int64_t)row * ld;
        int4 lo = *reinterpret_cast<const int4 *>(cp + tx * 4);
        int4 hi = *reinterpret_cast<const int4 *>(cp + 64 + tx * 4);
        acc[m][0] = lo.x; acc[m][1] = lo.y; acc[m][2] = lo.z; acc[m][3] = lo.w;
        acc[m][4] = hi.x; acc[m][5] = hi.y; acc[m][6] = hi.z; acc[m][7] = hi.w;
    }
    // chunk loaders: A chunk = rows 0..127, cols kc..kc+31 (1024 int4);
    //                B chunk = rows kc..kc+31, cols 0..127 (1024 int4)
    int4 pa[4], pb[4];
    auto load_chunk = [&](int kc) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            int idx = tid + 256 * q;
            int arow = idx >> 3, ac4 = idx & 7;
            pa[q] = *reinterpret_cast<const int4 *>(At + (int64_t)arow * ld + kc + ac4 * 4);
            int brow = idx >> 5, bc4 = idx & 31;
            pb[q] = *reinterpret_cast<const int4 *>(Bt + (int64_t)(kc + brow) * ld + bc4 * 4);
        }
    };
    auto store_chunk = [&]() {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            int idx = tid + 256 * q;
            int arow = idx >> 3, ac4 = idx & 7;
            As[ac4 * 4 + 0][arow] = (uint32_t)pa[q].x;
            As[ac4 * 4 + 1][arow] = (uint32_t)pa[q].y;
            As[ac4 * 4 + 2][arow] = (uint32_t)pa[q].z;
            As[ac4 * 4 + 3][arow] = (uint32_t)pa[q].w;
            int brow = idx >> 5, bc4 = idx & 31;
            *reinterpret_cast<int4 *>(&Bs[brow][bc4 * 4]) = pb[q];
        }
    };
    load_chunk(0);
    for (int kc = 0; kc < TILE; kc += KC) {
        __syncthreads();  // previous chunk fully consumed
        store_chunk();
        __syncthreads();
        if (kc + KC < TILE) load_chunk(kc + KC);  // overlaps with the compute below
#pragma unroll 1
        for (int k = 0; k < KC; k += 2) {
            uint4 a0l = *reinterpret_cast<const uint4 *>(&As[k][ty * 4]);
            uint4 a0h = *reinterpret_cast<const uint4 *>(&As[k][64 + ty * 4]);
            uint4 b0l = *reinterpret_cast<const uint4 *>(&Bs[k][tx * 4]);
            uint4 b0h = *reinterpret_cast<const uint4 *>(&Bs[k][64 + tx * 4]);
            uint4 a1l = *reinterpret_cast<const uint4 *>(&As[k + 1][ty * 4]);
            uint4 a1h = *reinterpret_cast<const uint4 *>(&As[k + 1][64 + ty * 4]);
            uint4 b1l = *reinterpret_cast<const uint4 *>(&Bs[k + 1][tx * 4]);
            uint4 b1h = *reinterpret_cast<const uint4 *>(&Bs[k + 1][64 + tx * 4]);
            uint32_t a0[8] = {a0l.x, a0l.y, a0l.z, a0l.w, a0h.x, a0h.y, a0h.z, a0h.w};
            uint32_t b0[8] = {b0l.x, b0l.y, b0l.z, b0l.w, b0h.x, b0h.y, b0h.z, b0h.w};
            uint32_t a1[8] = {a1l.x, a1l.y, a1l.z, a1l.w, a1h.x, a1h.y, a1h.z, a1h.w};
            uint32_t b1[8] = {b1l.x, b1l.y, b1l.z, b1l.w, b1h.x, b1h.y, b1h.z, b1h.w};
#pragma unroll
            for (int m = 0; m < 8; ++m)
#pragma unroll
                for (int c = 0; c < 8; ++c) acc[m][c] = umin3(acc[m][c], cat(a0[m], b0[c]), cat(a1[m], b1[c]));
        }
    }
    if (close) {
        // C := closure of C (the next round's pivot block, phase 1), on the
        // micro-tiles in registers.  Pivot k = 64 h + 4 g + e is row m = 4 h + e
        // of the threads with ty == g and column c = 4 h + e of those with
        // tx == g; they publish it to LDS, then every thread relaxes through
        // it.  Row k and column k do not change during pivot k.
        uint32_t *rowbuf = &As[0][0];  // rowbuf[j] = C[k][j]
        uint32_t *colbuf = &As[1][0];  // colbuf[i] = C[i][k]
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            for (int g = 0; g < 16; ++g) {
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    __syncthreads();  // the previous pivot's reads are done
                    if (ty == g) {
                        *reinterpret_cast<uint4 *>(&rowbuf[tx * 4]) = make_uint4(
                            acc[4 * h + e][0], acc[4 * h + e][1], acc[4 * h + e][2], acc[4 * h + e][3]);
                        *reinterpret_cast<uint4 *>(&rowbuf[64 + tx * 4]) = make_uint4(
                            acc[4 * h + e][4], acc[4 * h + e][5], acc[4 * h + e][6], acc[4 * h + e][7]);
                    }
                    if (tx == g) {
                        *reinterpret_cast<uint4 *>(&colbuf[ty * 4]) = make_uint4(
                            acc[0][4 * h + e], acc[1][4 * h + e], acc[2][4 * h + e], acc[3][4 * h + e]);
                        *reinterpret_cast<uint4 *>(&colbuf[64 + ty * 4]) = make_uint4(
                            acc[4][4 * h + e], acc[5][4 * h + e], acc[6][4 * h + e], acc[7][4 * h + e]);
                    }
                    __syncthreads();
                    const uint4 rl = *reinterpret_cast<const uint4 *>(&rowbuf[tx * 4]);
                    const uint4 rh = *reinterpret_cast<const uint4 *>(&rowbuf[64 + tx * 4]);
                    const uint4 cl = *reinterpret_cast<const uint4 *>(&colbuf[ty * 4]);
                    const uint4 ch = *reinterpret_cast<const uint4 *>(&colbuf[64 + ty * 4]);
                    const uint32_t rk[8] = {rl.x, rl.y, rl.z, rl.w, rh.x, rh.y, rh.z, rh.w};
                    const uint32_t ck[8] = {cl.x, cl.y, cl.z, cl.w, ch.x, ch.y, ch.z, ch.w};
#pragma unroll
                    for (int m = 0; m < 8; ++m)
#pragma unroll
                        for (int c = 0; c < 8; ++c) acc[m][c] = min(acc[m][c], cat(ck[m], rk[c]));
                }
            }
        }
    }
#pragma unroll
    for (int m = 0; m < 8; ++m) {
        int row = (m < 4) ? (ty * 4 + m) : (64 + ty * 4 + (m - 4));
        int32_t *cp = Ct + (int64_t)row * ld;
        *reinterpret_cast<int4 *>(cp + tx * 4) =
            make_int4((int)acc[m][0], (int)acc[m][1], (int)acc[m][2], (int)acc[m][3]);
        *reinterpret_cast<int4 *>(cp + 64 + tx * 4) =
            make_int4((int)acc[m][4], (int)acc[m][5], (int)acc[m][6], (int)acc[m][7]);
    }
}

// Phase 2: blocks [0, nb-1) are the row panel, [nb-1, 2(nb-1)) the column panel.
__global__ __launch_bounds__(256) void k_fw_panel(int32_t *D, int64_t ld, int32_t r, int32_t nb) {
    __shared__ uint32_t As[KC][LDS_W];
    __shared__ uint32_t Bs[KC][LDS_W];
    int32_t b = blockIdx.x;
    int32_t *P = D + (int64_t)r * TILE * ld + (int64_t)r * TILE;
    if (b < nb - 1) {
        int32_t j = b + (b >= r);
        int32_t *C = D + (int64_t)r * TILE * ld + (int64_t)j * TILE;
        minplus_tile(P, C, C, ld, As, Bs);
    } else {
        b -= nb - 1;
        int32_t i = b + (b >= r);
        int32_t *C = D + (int64_t)i * TILE * ld + (int64_t)r * TILE;
        minplus_tile(C, P, C, ld, As, Bs);
    }
}

// Phase 3: (nb-1)^2 tiles.  Work-groups are dealt round-robin to the 8 XCDs;
// the remap gives each XCD a contiguous run of tiles (same tile row i), so
// the column-panel tile D[i][r] is reused from that XCD's L2.
// With close_next, tile (r+1, r+1) -- the next round's pivot block, which no
// other work-group of this round reads -- goes to work-group 0 (dispatched
// first) and is closed there right after its update: the next round's
// phase 1 then runs under this round's phase 3 instead of as a launch of its
// own.
__global__ __launch_bounds__(256, 3) void k_fw_tiles(int32_t *D, int64_t ld, int32_t r, int32_t nb, int32_t close_next) {
    __shared__ uint32_t As[KC][LDS_W];
    __shared__ uint32_t Bs[KC][LDS_W];
    const int32_t m = nb - 1;
    const int32_t total = m * m;
    int32_t b = blockIdx.x;
    const int32_t per = total / 8;
    if (b < per * 8) b = (b & 7) * per + (b >> 3);
    const int32_t next = r * m + r;  // tile (r+1, r+1) with row and column r skipped
    if (close_next) b = b == next ? 0 : b == 0 ? next : b;
    int32_t ii = b / m, jj = b - ii * m;
    int32_t i = ii + (ii >= r), j = jj + (jj >= r);
    const int32_t *Ap = D + (int64_t)i * TILE * ld + (int64_t)r * TILE;
    const int32_t *Bp = D + (int64_t)r * TILE * ld + (int64_t)j * TILE;
    int32_t *C = D + (int64_t)i * TILE * ld + (int64_t)j * TILE;
    minplus_tile(Ap, Bp, C, ld, As, Bs, close_next && b == next);
}

const char *launch_fw(const DevGraph &g, int32_t n, hipStream_t s, Prof *prof) {
    if (n <= 0) return nullptr;
    const int32_t nb = (n + TILE - 1) / TILE;
    // round 0's pivot block on its own; every later one inside the previous
    // round's phase 3
    if (prof) prof->begin(KID_FW_PIVOT);
    k_fw_pivot<<<1, 1024, 0, s>>>(g.D, g.ld, 0);
    if (prof) prof->end();
    if (hipGetLastError() != hipSuccess) return "fw_pivot";
    for (int32_t r = 0; r < nb; ++r) {
        if (nb > 1) {
            if (prof) prof->begin(KID_FW_PANEL);
            k_fw_panel<<<2 * (nb - 1), 256, 0, s>>>(g.D, g.ld, r, nb);
            if (prof) prof->end();
            if (hipGetLastError() != hipSuccess) return "fw_panel";
            if (prof) prof->begin(KID_FW_TILE);
            k_fw_tiles<<<(nb - 1) * (nb - 1), 256, 0, s>>>(g.D, g.ld, r, nb, r + 1 < nb ? 1 : 0);
            if (prof) prof->end();
            if (hipGetLastError() != hipSuccess) return "fw_tiles";
        }
    }
    return nullptr;
}

APSP_SR_END
}  // namespace apsp
