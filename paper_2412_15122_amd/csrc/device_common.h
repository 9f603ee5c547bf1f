// Device helpers shared by the library's kernels (wave64, 256-thread blocks).
#pragma once
#include "apsp_internal.h"

namespace apsp {
APSP_SR_BEGIN

// ---------------------------------------------------------------------------
// wave / block helpers (wave64)
// ---------------------------------------------------------------------------

__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }

// A 16-byte load marked non-temporal: a sweep reads each entry of D once per
// launch, so the line need not stay in the caches.
__device__ __forceinline__ uint4 load_stream4(const int32_t *p) {
    typedef unsigned int v4u __attribute__((ext_vector_type(4)));
    const v4u t = __builtin_nontemporal_load(reinterpret_cast<const v4u *>(p));
    return make_uint4(t.x, t.y, t.z, t.w);
}

__device__ __forceinline__ uint32_t wave_min(uint32_t v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = min(v, (uint32_t)__shfl_xor((int)v, o));
    return v;
}

__device__ __forceinline__ uint32_t wave_max(uint32_t v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = max(v, (uint32_t)__shfl_xor((int)v, o));
    return v;
}

// min(bound, min over x < n of a[x] (+) b[x]) (uint32; entries <= INF, a >=
// 0), by one wavefront: b is read in full (16-byte loads, four per lane in
// flight), a only where b[x] < bound (no other x can go below bound).
// a and b 16-byte aligned.
__device__ inline uint32_t wave_min_plus_below(const int32_t *a, const int32_t *b, int32_t n, uint32_t bound) {
    const int lane = lane_id();
    uint32_t best = bound;
    const int32_t n4 = n & ~3;
    for (int32_t base = 0; base < n4; base += 1024) {
        uint4 vb[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int32_t x = base + (q * 64 + lane) * 4;
            vb[q] = make_uint4(INF, INF, INF, INF);
            if (x < n4) vb[q] = *reinterpret_cast<const uint4 *>(b + x);
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int32_t x = base + (q * 64 + lane) * 4;
            const uint32_t w[4] = {vb[q].x, vb[q].y, vb[q].z, vb[q].w};
#pragma unroll
            for (int e = 0; e < 4; ++e)
                if (w[e] < best) best = min(best, cat((uint32_t)a[x + e], w[e]));
        }
    }
    if (n4 + lane < n) {
        const uint32_t w = (uint32_t)b[n4 + lane];
        if (w < best) best = min(best, cat((uint32_t)a[n4 + lane], w));
    }
    return wave_min(best);
}

// min over x < n of a[x] (+) b[x] (uint32; entries <= INF), by one wavefront:
// 16-byte loads (a and b 16-byte aligned), four of each per lane in flight.
__device__ inline uint32_t wave_min_plus(const int32_t *a, const int32_t *b, int32_t n) {
    const int lane = lane_id();
    uint32_t best = INF;
    const int32_t n4 = n & ~3;
    for (int32_t base = 0; base < n4; base += 1024) {
        uint4 va[4], vb[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int32_t x = base + (q * 64 + lane) * 4;
            va[q] = make_uint4(INF, INF, INF, INF);
            vb[q] = va[q];
            if (x < n4) {
                va[q] = *reinterpret_cast<const uint4 *>(a + x);
                vb[q] = *reinterpret_cast<const uint4 *>(b + x);
            }
        }
#pragma unroll
        for (int q = 0; q < 4; ++q)
            best = min(min(best, min(cat(va[q].x, vb[q].x), cat(va[q].y, vb[q].y))),
                       min(cat(va[q].z, vb[q].z), cat(va[q].w, vb[q].w)));
    }
    if (n4 + lane < n) best = min(best, cat((uint32_t)a[n4 + lane], (uint32_t)b[n4 + lane]));
    return wave_min(best);
}

__device__ __forceinline__ int wave_sum(int v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// Block-wide reductions for 256 threads; `red` holds >= 4 words of LDS.
__device__ inline uint32_t block_min256(uint32_t v, uint32_t *red) {
    v = wave_min(v);
    __syncthreads();
    if (lane_id() == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    uint32_t r = min(min(red[0], red[1]), min(red[2], red[3]));
    return r;
}

__device__ inline int block_sum256(int v, uint32_t *red) {
    v = wave_sum(v);
    __syncthreads();
    if (lane_id() == 0) red[threadIdx.x >> 6] = (uint32_t)v;
    __syncthreads();
    return (int)(red[0] + red[1] + red[2] + red[3]);
}

// Exclusive prefix sum over the 256 threads of a block; returns this thread's
// offset and writes the total to *total.  `red` holds >= 8 words.
__device__ inline int block_exscan256(int v, uint32_t *red, int *total) {
    const int lane = lane_id(), wid = threadIdx.x >> 6;
    int incl = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        int t = __shfl_up(incl, o);
        if (lane >= o) incl += t;
    }
    __syncthreads();
    if (lane == 63) red[wid] = (uint32_t)incl;
    __syncthreads();
    int base = 0;
    for (int w = 0; w < wid; ++w) base += (int)red[w];
    *total = (int)(red[0] + red[1] + red[2] + red[3]);
    return base + incl - v;
}

// Block-wide reductions for NT threads (a multiple of 64); `red` holds at
// least NT / 64 words of LDS.
template <int NT>
__device__ inline uint32_t block_min(uint32_t v, uint32_t *red) {
    v = wave_min(v);
    __syncthreads();
    if (lane_id() == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    uint32_t r = red[0];
#pragma unroll
    for (int w = 1; w < NT / 64; ++w) r = min(r, red[w]);
    return r;
}

template <int NT>
__device__ inline int block_sum(int v, uint32_t *red) {
    v = wave_sum(v);
    __syncthreads();
    if (lane_id() == 0) red[threadIdx.x >> 6] = (uint32_t)v;
    __syncthreads();
    int r = 0;
#pragma unroll
    for (int w = 0; w < NT / 64; ++w) r += (int)red[w];
    return r;
}

template <int NT>
__device__ inline int block_exscan(int v, uint32_t *red, int *total) {
    const int lane = lane_id(), wid = threadIdx.x >> 6;
    int incl = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        int t = __shfl_up(incl, o);
        if (lane >= o) incl += t;
    }
    __syncthreads();
    if (lane == 63) red[wid] = (uint32_t)incl;
    __syncthreads();
    int base = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < NT / 64; ++w) {
        base += w < wid ? (int)red[w] : 0;
        tot += (int)red[w];
    }
    *total = tot;
    return base + incl - v;
}

struct SelectShared {
    uint32_t hist[256];
    uint32_t red[32];
    int bin, kk;
    unsigned long long keys[NIN_L];
};

// Select the NIN_L smallest entries of vals[0..n) other than index `excl`
// and other than INF (absent edges), ordered by (w, x).  One block of NT
// threads; `stage` is LDS for n words (the values are read from memory once).
template <int NT = 256>
__device__ inline void select_light(const int32_t *__restrict__ vals, int32_t n, int32_t excl, int2 *list,
                             int32_t *cnt_out, int32_t *beta_out, SelectShared &sh, uint32_t *stage) {
    const int tid = threadIdx.x;
    int valid = 0;
    uint32_t tmin = INF;  // this thread's smallest staged value
    // stage the values: 16-byte loads, four per thread in flight (scalar
    // loads for a misaligned vector and the tail)
    const int32_t n4 = ((uintptr_t)vals & 15) ? 0 : (n & ~3);
    for (int32_t base = 0; base < n4; base += NT * 16) {
        uint4 v[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int32_t x = base + (q * NT + tid) * 4;
            if (x < n4) v[q] = *reinterpret_cast<const uint4 *>(vals + x);
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int32_t x = base + (q * NT + tid) * 4;
            if (x < n4) {
                uint4 u = v[q];
                if ((uint32_t)(excl - x) < 4u) {
                    const int e = excl - x;
                    if (e == 0) u.x = INF;
                    if (e == 1) u.y = INF;
                    if (e == 2) u.z = INF;
                    if (e == 3) u.w = INF;
                }
                stage[x] = u.x;  // (the LDS stage is only 4-byte aligned)
                stage[x + 1] = u.y;
                stage[x + 2] = u.z;
                stage[x + 3] = u.w;
                valid += (u.x < INF) + (u.y < INF) + (u.z < INF) + (u.w < INF);
                tmin = min(tmin, min(min(u.x, u.y), min(u.z, u.w)));
            }
        }
    }
    for (int32_t x = n4 + tid; x < n; x += NT) {
        uint32_t v = (uint32_t)vals[x];
        if (x == excl) v = INF;
        stage[x] = v;
        valid += v < INF;
        tmin = min(tmin, v);
    }
    int total = block_sum<NT>(valid, sh.red);
    uint32_t tau = INF;  // entries < tau are all taken
    int need_eq = 0;     // plus this many entries == tau, lowest index first
    // Finds the bin holding rank kk of sh.hist; writes sh.bin and sh.kk.
    auto find_bin = [&](int kk) {
        if (tid < 64) {
            const uint32_t h0 = sh.hist[4 * tid], h1 = sh.hist[4 * tid + 1], h2 = sh.hist[4 * tid + 2],
                           h3 = sh.hist[4 * tid + 3];
            const int own = (int)(h0 + h1 + h2 + h3);
            int incl = own;
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
                const int t = __shfl_up(incl, o);
                if (tid >= o) incl += t;
            }
            const int before = incl - own;
            if (before < kk && kk <= incl) {
                int cum = before, b = 4 * tid;
                const uint32_t hh[4] = {h0, h1, h2, h3};
                for (int q = 0; q < 3; ++q, ++b) {
                    if (cum + (int)hh[q] >= kk) break;
                    cum += (int)hh[q];
                }
                sh.bin = b;
                sh.kk = kk - cum;
            }
            if (tid == 63 && incl < kk) sh.bin = -1;  // rank beyond the histogram
        }
        __syncthreads();
    };
    if (total > NIN_L) {
        // light weights are usually packed near the minimum: try the 256
        // values [vmin, vmin + 256) first (one histogram, few collisions)
        const uint32_t vmin = block_min<NT>(tmin, sh.red);
        if (tid < 256) sh.hist[tid] = 0;
        __syncthreads();
        for (int32_t x = tid; x < n; x += NT) {
            const uint32_t w = stage[x];
            if (w < INF && w - vmin < 256u) atomicAdd(&sh.hist[w - vmin], 1u);
        }
        __syncthreads();
        find_bin(NIN_L);
        if (sh.bin >= 0) {
            tau = vmin + (uint32_t)sh.bin;
            need_eq = sh.kk;
        } else {
            uint32_t prefix = 0, mask = 0;
            int kk = NIN_L;
            for (int shift = 24; shift >= 0; shift -= 8) {
                __syncthreads();
                if (tid < 256) sh.hist[tid] = 0;
                __syncthreads();
                for (int32_t x = tid; x < n; x += NT) {
                    const uint32_t v = stage[x];
                    if (v < INF && (v & mask) == prefix) atomicAdd(&sh.hist[(v >> shift) & 255u], 1u);
                }
                __syncthreads();
                find_bin(kk);
                prefix |= (uint32_t)sh.bin << shift;
                mask |= 255u << shift;
                kk = sh.kk;
            }
            tau = prefix;
            need_eq = kk;
        }
        __syncthreads();
    }
    // ordered collection: wavefront w takes the contiguous range [w span,
    // (w + 1) span) and reads it 64 consecutive values at a time (no LDS bank
    // conflicts); ballots rank the kept entries in index order
    constexpr int NWAVES = NT / 64;
    const int wid = tid >> 6, lane = tid & 63;
    const unsigned long long below = (1ull << lane) - 1ull;
    const int32_t span = (((n + NWAVES - 1) / NWAVES) + 63) & ~63;
    const int32_t xa = min(n, wid * span), xb = min(n, xa + span);
    int c_less = 0, c_eq = 0;  // this wavefront's counts
    for (int32_t b = xa; b < xb; b += 64) {  // wave-uniform
        const int32_t x = b + lane;
        const uint32_t v = x < xb ? stage[x] : INF;
        c_less += __popcll(__ballot(v < tau));
        c_eq += __popcll(__ballot(v == tau && v < INF));
    }
    __syncthreads();
    if (lane == 0) {
        sh.red[wid] = (uint32_t)c_less;
        sh.red[16 + wid] = (uint32_t)c_eq;
    }
    __syncthreads();
    int off_less = 0, off_eq = 0, tot_less = 0;
#pragma unroll
    for (int w = 0; w < NWAVES; ++w) {
        const int a = (int)sh.red[w], e = (int)sh.red[16 + w];
        if (w < wid) {
            off_less += a;
            off_eq += e;
        }
        tot_less += a;
    }
    for (int32_t b = xa; b < xb; b += 64) {  // wave-uniform
        const int32_t x = b + lane;
        const uint32_t v = x < xb ? stage[x] : INF;
        const unsigned long long ml = __ballot(v < tau), me = __ballot(v == tau && v < INF);
        if (v < tau) {
            sh.keys[off_less + __popcll(ml & below)] = ((unsigned long long)v << 32) | (uint32_t)x;
        } else if (v == tau && v < INF) {
            const int r = off_eq + __popcll(me & below);
            if (r < need_eq) sh.keys[tot_less + r] = ((unsigned long long)v << 32) | (uint32_t)x;
        }
        off_less += __popcll(ml);
        off_eq += __popcll(me);
    }
    __syncthreads();
    const int m = min(total, NIN_L);
    if (tid < 64) {  // bitonic sort of 64 keys in one wave
        const int lane = tid;
        unsigned long long key = lane < m ? sh.keys[lane] : ~0ull;
        for (int k = 2; k <= 64; k <<= 1) {
            for (int j = k >> 1; j > 0; j >>= 1) {
                uint32_t lo = (uint32_t)key, hi = (uint32_t)(key >> 32);
                uint32_t olo = (uint32_t)__shfl_xor((int)lo, j), ohi = (uint32_t)__shfl_xor((int)hi, j);
                unsigned long long other = ((unsigned long long)ohi << 32) | olo;
                bool up = (lane & k) == 0;
                bool lower = (lane & j) == 0;
                unsigned long long mn = key < other ? key : other;
                unsigned long long mx = key < other ? other : key;
                key = (lower == up) ? mn : mx;
            }
        }
        int2 ent;
        if (lane < m) {
            ent.x = (int32_t)(uint32_t)key;
            ent.y = (int32_t)(uint32_t)(key >> 32);
        } else {
            ent.x = 0;
            ent.y = (int32_t)INF;
        }
        list[lane] = ent;
        if (lane == 0) {
            *cnt_out = m;
            *beta_out = (int32_t)(total > NIN_L ? tau : INF);
        }
    }
    __syncthreads();
}

// Wave-level list edits (one wave owns list y).
__device__ inline void wave_list_purge(const DevGraph &g, int32_t y, int32_t x) {
    const int lane = lane_id();
    int2 *L = g.nin + (int64_t)y * NIN_L;
    const int cnt = g.nin_cnt[y];
    int2 ent = lane < cnt ? L[lane] : make_int2(0, (int)INF);
    unsigned long long m = __ballot(lane < cnt && ent.x == x);
    if (m == 0) return;
    const int pos = __ffsll((long long)m) - 1;
    int nx = __shfl_down(ent.x, 1), ny = __shfl_down(ent.y, 1);
    if (lane >= pos && lane < cnt - 1) L[lane] = make_int2(nx, ny);
    if (lane == cnt - 1) L[lane] = make_int2(0, (int)INF);
    if (lane == 0) g.nin_cnt[y] = cnt - 1;
}

// Insert in-edge (x, w) into list y if w < beta (dropping the heaviest entry
// when full and lowering beta to it).  Caller guarantees x is not listed.
__device__ inline void wave_list_insert(const DevGraph &g, int32_t y, int32_t x, uint32_t w) {
    const int lane = lane_id();
    int2 *L = g.nin + (int64_t)y * NIN_L;
    const int cnt = g.nin_cnt[y];
    const uint32_t beta = (uint32_t)g.nin_beta[y];
    if (w >= INF || w >= beta) return;
    int2 ent = lane < cnt ? L[lane] : make_int2(0, (int)INF);
    const int pos = __popcll(__ballot(lane < cnt && (uint32_t)ent.y <= w));
    int px = __shfl_up(ent.x, 1), py = __shfl_up(ent.y, 1);
    const int ncnt = min(cnt + 1, NIN_L);
    uint32_t dropped = INF;
    if (cnt == NIN_L) dropped = (pos < NIN_L) ? (uint32_t)__shfl(ent.y, NIN_L - 1) : w;
    int2 ne = lane < pos ? ent : (lane == pos ? make_int2(x, (int)w) : make_int2(px, py));
    if (lane < ncnt) L[lane] = ne;
    if (lane == 0) {
        g.nin_cnt[y] = ncnt;
        if (cnt == NIN_L) g.nin_beta[y] = (int32_t)min(beta, dropped);
    }
}

__device__ inline void wave_list_set_edge(const DevGraph &g, int32_t y, int32_t x, uint32_t w) {
    wave_list_purge(g, y, x);
    wave_list_insert(g, y, x, w);
}

// Minimum over a group of 16 lanes (xor offsets below 16 stay in the group).
__device__ __forceinline__ uint32_t group16_min(uint32_t v) {
#pragma unroll
    for (int o = 8; o > 0; o >>= 1) v = min(v, (uint32_t)__shfl_xor((int)v, o, 16));
    return v;
}

constexpr int FUSED_UNROLL = 4;  // int4 loads in flight per thread and row
constexpr int LDS_LIST = 128;    // flagged columns a block-per-row recompute keeps in LDS

__device__ __forceinline__ unsigned long long lanes_below() {
    return (1ull << lane_id()) - 1ull;
}

struct FusedShared {
    uint32_t *cur, *fl, *fl2, *red, *flag_changed, *flag_nfs;
    int32_t *list_lds;
};

__device__ inline FusedShared fused_shared(const DevGraph &g, uint32_t *sm) {
    FusedShared f;
    const int nwp = (g.P + 31) >> 5;
    f.cur = sm;
    f.fl = sm + g.P;
    f.fl2 = f.fl + nwp;
    f.list_lds = (int32_t *)(f.fl2 + nwp);
    f.red = (uint32_t *)(f.list_lds + LDS_LIST);
    f.flag_changed = f.red + 32;
    f.flag_nfs = f.red + 33;
    return f;
}

// The pair tests of row i (block-uniform).
struct RowTests {
    bool t1, t2;
    uint32_t a1, a2;
};

__device__ inline RowTests row_tests(const DevGraph &g, const FusedArgs &fa, int32_t i, uint32_t w_old) {
    RowTests r{false, false, 0, 0};
    if (fa.mode == FUSED_REMOVE) {
        const uint32_t dik = (uint32_t)fa.col1[i];
        r.t1 = (i != fa.k) && dik < INF;
        r.a1 = dik;
    } else {
        const uint32_t cu = (uint32_t)fa.col1[i], cv = (uint32_t)fa.col2[i];
        r.t1 = cv < INF && cat(cu, w_old) == cv;
        r.a1 = cv;
        if (g.undirected) {
            r.t2 = cu < INF && cat(cv, w_old) == cu;
            r.a2 = cu;
        }
    }
    return r;
}

// The value D[i][y] had before the update, for a flagged y of row i: the
// pair test that flagged it holds with equality (removal: D[i][k] + D[k][y];
// increase: D[i][u] + w_old + D[v][y], or the swapped term when undirected).
// A recomputed entry can only go up from here, so an entry back at this value
// is final, and one above it belongs to the refined set (Theorem
// Theorem 6: every shortest path of that pair used k, or the edge).
__device__ inline uint32_t flagged_old(const FusedArgs &fa, const RowTests &rt, int32_t y) {
    const uint32_t o1 = rt.t1 ? cat(rt.a1, (uint32_t)fa.row1[y]) : INF;
    const uint32_t o2 = rt.t2 ? cat(rt.a2, (uint32_t)fa.row2[y]) : INF;
    return min(o1, o2);
}

// Mask pass over row i.  Each lane tests 4 consecutive columns; 8 lanes
// assemble a 32-bit flag word with shuffles (no clearing, no atomics).
//   fill == 0: cur[j] = INF for flagged j, D[i][j] otherwise (fl = flags)
//   fill == 1: (heavy-row pass) flagged j whose row is light takes the
//              mirrored D[j][i]; flagged j whose row is heavy (heavy[j] ==
//              epoch) is INF and goes to fl2; fl = all flags.
// Returns this thread's flag count.
__device__ inline int mask_row(const DevGraph &g, const FusedArgs &fa, int32_t i, const RowTests &rt, FusedShared &sh,
                        bool write_cur, int fill) {
    const int n = g.n_slots;
    const int tid = threadIdx.x, lane = lane_id();
    const int32_t *Drow = g.D + (int64_t)i * g.ld;
    int cnt = 0;
    // the trip count is block-uniform: the shuffles below need every lane
    for (int b = 0; b * 4 < n; b += FUSED_THREADS * FUSED_UNROLL) {
        const int q0 = b + tid;
        uint4 d[FUSED_UNROLL], r1[FUSED_UNROLL], r2[FUSED_UNROLL];
#pragma unroll
        for (int u = 0; u < FUSED_UNROLL; ++u) {
            const int j0 = (q0 + u * FUSED_THREADS) * 4;
            d[u] = make_uint4(INF, INF, INF, INF);
            r1[u] = r2[u] = make_uint4(0, 0, 0, 0);
            if (j0 < n) {
                d[u] = *reinterpret_cast<const uint4 *>(Drow + j0);
                if (rt.t1) r1[u] = *reinterpret_cast<const uint4 *>(fa.row1 + j0);
                if (rt.t2) r2[u] = *reinterpret_cast<const uint4 *>(fa.row2 + j0);
            }
        }
#pragma unroll
        for (int u = 0; u < FUSED_UNROLL; ++u) {
            const int j0 = (q0 + u * FUSED_THREADS) * 4;
            const uint32_t dv[4] = {d[u].x, d[u].y, d[u].z, d[u].w};
            const uint32_t v1[4] = {r1[u].x, r1[u].y, r1[u].z, r1[u].w};
            const uint32_t v2[4] = {r2[u].x, r2[u].y, r2[u].z, r2[u].w};
            uint32_t bits = 0, hbits = 0;
            uint32_t cv[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int j = j0 + e;
                uint32_t dj = dv[e];
                bool f = false;
                if (j < n && j != i && dj < INF)
                    f = (rt.t1 && cat(rt.a1, v1[e]) == dj) || (rt.t2 && cat(rt.a2, v2[e]) == dj);
                if (fa.mode == FUSED_REMOVE && j == fa.k) {
                    f = false;
                    dj = INF;
                }
                bits |= (uint32_t)f << e;
                cv[e] = dj;
                if (f) {
                    if (fill == 1 && fa.heavy_epoch[j] != fa.epoch) {
                        cv[e] = (uint32_t)g.D[(int64_t)j * g.ld + i];
                    } else {
                        cv[e] = INF;
                        hbits |= 1u << e;
                    }
                }
            }
            cnt += __popc(bits);
            uint32_t word = bits << ((lane & 7) * 4);
            uint32_t hword = hbits << ((lane & 7) * 4);
#pragma unroll
            for (int o = 1; o < 8; o <<= 1) {
                word |= (uint32_t)__shfl_xor((int)word, o);
                hword |= (uint32_t)__shfl_xor((int)hword, o);
            }
            if (j0 < n) {
                if (write_cur) *reinterpret_cast<uint4 *>(sh.cur + j0) = make_uint4(cv[0], cv[1], cv[2], cv[3]);
                if ((lane & 7) == 0) {
                    sh.fl[j0 >> 5] = word;
                    if (fill == 1) sh.fl2[j0 >> 5] = hword;
                }
            }
        }
    }
    return cnt;
}

// Bitmap words -> ascending column list (block-wide); returns the count.
__device__ inline int compact_bits(const uint32_t *bm, int nw, int32_t *list, uint32_t *red) {
    const int tid = threadIdx.x;
    const int per = (nw + FUSED_THREADS - 1) / FUSED_THREADS;
    const int w0 = min(nw, tid * per), w1 = min(nw, w0 + per);
    int c = 0;
    for (int w = w0; w < w1; ++w) c += __popc(bm[w]);
    int tot;
    int off = block_exscan<FUSED_THREADS>(c, red, &tot);
    for (int w = w0; w < w1; ++w) {
        uint32_t bits = bm[w];
        while (bits) {
            const int b = __ffs(bits) - 1;
            bits &= bits - 1;
            list[off++] = w * 32 + b;
        }
    }
    __syncthreads();
    return tot;
}

// Index entries e and e+1 of a node's light in-edge list as (x, w, x', w');
// entries at or past lim read as weight INF.
__device__ __forceinline__ int4 index_pair(const int4 *L4, int lim, int e) {
    int4 p = make_int4(0, (int)INF, 0, (int)INF);
    if (e < lim) p = L4[e >> 1];
    if (e + 1 >= lim) p.w = (int)INF;
    return p;
}

// cm lowered by row[x] (+) w for the pair's edges lighter than best (row:
// a row of D in global memory, or its copy in LDS).
template <class T>
__device__ __forceinline__ uint32_t pull_pair(const T *row, int4 p, uint32_t best, uint32_t cm) {
    if ((uint32_t)p.y < best) cm = min(cm, cat((uint32_t)row[p.x], (uint32_t)p.y));
    if ((uint32_t)p.w < best) cm = min(cm, cat((uint32_t)row[p.z], (uint32_t)p.w));
    return cm;
}

// Minimum over an aligned group of four lanes.
__device__ __forceinline__ uint32_t group4_min(uint32_t v) {
    v = min(v, (uint32_t)__shfl_xor((int)v, 1, 4));
    return min(v, (uint32_t)__shfl_xor((int)v, 2, 4));
}

// Bellman-Ford relaxation of the columns list[0..total) of the LDS row cur:
//   cur[y] = min_x cur[x] (+) A'[x][y]
// Sweeps scan each y's light in-edges (4 lanes per y, 32 entries per round
// trip, stopping once an entry is at least the current value; unused
// entries are (0, INF) sentinels).  When the sweeps are stable, every y
// above its index bound beta gets an exhaustive scan of its in-edges, and
// the sweeps resume if that changed anything.
__device__ inline void row_bellman_ford(const DevGraph &g, FusedShared &sh, const int32_t *list, int total, int32_t *fsl,
                                 int &sweeps, int &nfs_total) {
    const int n = g.n_slots;
    const int tid = threadIdx.x;
    const int grp = tid >> 2, l4 = tid & 3;
    constexpr int NG = FUSED_THREADS / 4;
    const int lim = g.lim;
    const int32_t *Min = in_matrix(g);
    uint32_t *cur = sh.cur;
    // each group's first column and its 32 lightest in-edges stay in
    // registers for all sweeps: a sweep over at most NG columns reads only LDS
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
            if (tid == 0) *sh.flag_changed = 0;
            __syncthreads();
            bool changed = false;
            if (has0) {
                uint32_t best = cur[y0];
                uint32_t cm = pull_pair(cur, q0, best, INF);
                cm = pull_pair(cur, q1, best, cm);
                cm = pull_pair(cur, q2, best, cm);
                cm = pull_pair(cur, q3, best, cm);
                best = min(best, group4_min(cm));
                for (int c0 = 32; c0 < lim && wl0 < best; c0 += 32) {  // rare: the rest from the index
                    uint32_t cr = INF;
#pragma unroll
                    for (int q = 0; q < 4; ++q) cr = pull_pair(cur, index_pair(Y4, lim, c0 + 8 * q + 2 * l4), best, cr);
                    best = min(best, group4_min(cr));
                    const uint32_t wl = (uint32_t)__shfl(index_pair(Y4, lim, c0 + 24 + 2 * l4).w, 3, 4);
                    if (wl >= best) break;
                }
                if (l4 == 0 && best < cur[y0]) {
                    cur[y0] = best;
                    changed = true;
                }
            }
            for (int e = grp + NG; e < total; e += NG) {
                const int32_t y = list[e];
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
                    if (wlast >= best) break;  // every later entry is at least as heavy
                }
                if (l4 == 0 && best < cur[y]) {
                    cur[y] = best;
                    changed = true;
                }
            }
            if (changed) *sh.flag_changed = 1;
            __syncthreads();
            ++sweeps;
            if (*sh.flag_changed == 0) break;
        }
        __syncthreads();
        if (tid == 0) *sh.flag_nfs = 0;
        __syncthreads();
        for (int e = tid; e < total; e += FUSED_THREADS) {
            const int32_t y = list[e];
            uint32_t beta_eff = (uint32_t)g.nin_beta[y];
            if (lim < NIN_L) beta_eff = min(beta_eff, (uint32_t)g.nin[(int64_t)y * NIN_L + lim].y);
            if (cur[y] > beta_eff) fsl[atomicAdd(sh.flag_nfs, 1u)] = y;
        }
        __syncthreads();
        const int nfs = (int)*sh.flag_nfs;
        if (nfs == 0) break;
        if (tid == 0) *sh.flag_changed = 0;
        for (int f = 0; f < nfs; ++f) {
            const int32_t y = fsl[f];
            const int32_t *col = Min + (int64_t)y * g.ld;
            uint32_t best = INF;
            for (int32_t x = tid; x < n; x += FUSED_THREADS) best = min(best, cat(cur[x], (uint32_t)col[x]));
            best = block_min<FUSED_THREADS>(best, sh.red);
            if (tid == 0 && best < cur[y]) {
                cur[y] = best;
                *sh.flag_changed = 1;
            }
            __syncthreads();
        }
        nfs_total += nfs;
        __syncthreads();
        if (*sh.flag_changed == 0) break;
    }
}

__device__ __forceinline__ uint32_t q_wave_min(uint32_t v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = min(v, (uint32_t)__shfl_xor((int)v, o));
    return v;
}

// Block-wide minimum of a 64-bit key for 1024 threads.
__device__ inline unsigned long long block_min_key(unsigned long long v, unsigned long long *red) {
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
// and j; by Theorem 5 they contain every shortest i -> j path.
// The walk takes, from cur, the candidate b with the smallest id such that
// A[cur][b] + D[b][j] == D[cur][j] (the edge starts a shortest path to j).
// With weights >= 1 this yields the lexicographically smallest shortest
// path.  Zero-weight edges can trap the greedy walk in a zero cycle; then a
// breadth-first search over the same tight edges returns a shortest simple
// path instead.
__device__ inline void query_block(const DevGraph &g, int32_t si, int32_t sj, int32_t *out, int32_t *scratch) {
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
        __syncthreads();
        return;
    }
    if (dist >= INF) {
        if (tid == 0) { out[0] = (int32_t)INF; out[1] = 0; out[2] = 0; }
        __syncthreads();
        return;
    }
    if (tid == 0) { s_k = 0; s_ci = -1; s_cj = -1; }
    for (int w = tid; w < (n + 31) / 32; w += blockDim.x) visited[w] = 0;
    __syncthreads();
    for (int32_t t = tid; t < n; t += blockDim.x) {
        if (g.id_of_slot[t] < 0) continue;
        const uint32_t dit = (uint32_t)g.D[(int64_t)si * ld + t];
        const uint32_t dtj = (uint32_t)g.D[(int64_t)t * ld + sj];
        if (t == si || t == sj || cat(dit, dtj) == dist) {
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
            if (cat(a, (uint32_t)candD[c]) == dcur) {
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
        __syncthreads();
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
                if (w < INF && cat(w, (uint32_t)candD[c2]) == (uint32_t)candD[c]) {
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
    __syncthreads();
}

// Smallest 64-bit key over a wavefront.
__device__ __forceinline__ unsigned long long wave_min_key(unsigned long long v) {
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)v, o);
        const uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)(v >> 32), o);
        const unsigned long long u = ((unsigned long long)hi << 32) | lo;
        v = u < v ? u : v;
    }
    return v;
}

// Bellman-Ford over the flagged columns list[0..cnt) of row Drow (in place),
// one wavefront: 16 groups of 4 lanes, each group one column at a time,
// reading 16 index entries per load and stopping once an entry is at least
// the current value.  Columns left above their index bound get exhaustive
// in-edge scans, and the sweeps resume if that changed anything.
__device__ inline void wave_bellman_ford(const DevGraph &g, int32_t *Drow, const int32_t *list, int cnt, int32_t *fsl,
                                  int &sweeps, int &nfs_total, const int32_t *olds = nullptr) {
    const int lane = lane_id();
    const int g4 = lane >> 2, l4 = lane & 3;
    const int lim = g.lim;
    const int n = g.n_slots;
    const int32_t *Min = in_matrix(g);
    for (;;) {
        for (;;) {
            bool changed = false;
            for (int e = g4; e < cnt; e += 16) {
                const int32_t y = list[e];
                uint32_t best = (uint32_t)Drow[y];
                // a lower bound: the old value when distances only go up
                // (an entry back at it is final), else 0
                const uint32_t floor = olds ? (uint32_t)olds[e] : 0u;
                if (best <= floor) continue;
                const int4 *L4 = reinterpret_cast<const int4 *>(g.nin + (int64_t)y * NIN_L);
                // lane l4 of the group holds entries 2*l4 + 8*q and the next,
                // q = 0..3: the lightest eight are gathered first, and the
                // rest only below the bound they give.  Most of the cost is
                // the random reads of D, so a scan gathers as few as it can.
                int4 p0 = index_pair(L4, lim, 2 * l4), p1 = index_pair(L4, lim, 8 + 2 * l4);
                int4 p2 = index_pair(L4, lim, 16 + 2 * l4), p3 = index_pair(L4, lim, 24 + 2 * l4);
                best = min(best, group4_min(pull_pair(Drow, p0, best, INF)));
                uint32_t wl = (uint32_t)__shfl(p0.w, 3, 4);  // the eighth entry
                for (int c0 = 32; best > floor && wl < best; c0 += 32) {
                    uint32_t cm = pull_pair(Drow, p1, best, INF);
                    cm = pull_pair(Drow, p2, best, cm);
                    cm = pull_pair(Drow, p3, best, cm);
                    best = min(best, group4_min(cm));
                    wl = (uint32_t)__shfl(p3.w, 3, 4);  // the last entry of this block of 32
                    if (c0 >= lim || best <= floor || wl >= best) break;
                    p0 = index_pair(L4, lim, c0 + 2 * l4);
                    p1 = index_pair(L4, lim, c0 + 8 + 2 * l4);
                    p2 = index_pair(L4, lim, c0 + 16 + 2 * l4);
                    p3 = index_pair(L4, lim, c0 + 24 + 2 * l4);
                    best = min(best, group4_min(pull_pair(Drow, p0, best, INF)));
                    wl = (uint32_t)__shfl(p0.w, 3, 4);
                }
                if (l4 == 0 && best < (uint32_t)Drow[y]) {
                    Drow[y] = (int32_t)best;
                    changed = true;
                }
            }
            __threadfence_block();
            ++sweeps;
            if (!__any(changed)) break;
        }
        int nfs = 0;
        for (int b = 0; b < cnt; b += 64) {
            const int e = b + lane;
            bool need = false;
            int32_t y = 0;
            if (e < cnt) {
                y = list[e];
                uint32_t beta_eff = (uint32_t)g.nin_beta[y];
                if (lim < NIN_L) beta_eff = min(beta_eff, (uint32_t)g.nin[(int64_t)y * NIN_L + lim].y);
                need = (uint32_t)Drow[y] > beta_eff && !(olds && Drow[y] == olds[e]);
            }
            const unsigned long long m = __ballot(need);
            if (need) fsl[nfs + __popcll(m & lanes_below())] = y;
            nfs += __popcll(m);
        }
        if (nfs == 0) break;
        bool changed = false;
        for (int f = 0; f < nfs; ++f) {
            const int32_t y = fsl[f];
            const int32_t *col = Min + (int64_t)y * g.ld;
            const uint32_t best = wave_min_plus(Drow, col, n);
            if (best < (uint32_t)Drow[y]) {
                changed = true;
                if (lane == 0) Drow[y] = (int32_t)best;
            }
            __threadfence_block();
        }
        nfs_total += nfs;
        if (!changed) break;
    }
}

// One wave: read the old weight and D[u][v], pick the path, write A, fix the
// index lists of v (and u).
//   w == w_old                      -> nothing changes
//   w <  w_old and w <  D[u][v]     -> decrease relaxation
//   w <  w_old and w >= D[u][v]     -> nothing changes in D
//   w >  w_old and w_old == D[u][v] -> increase: mask + recompute
//   w >  w_old and w_old >  D[u][v] -> the edge is on no shortest path
__device__ inline void edge_begin_wave(const DevGraph &g, int32_t su, int32_t sv, int32_t w) {
    const int lane = lane_id();
    const int64_t ld = g.ld;
    const uint32_t w_old = (uint32_t)g.A[(int64_t)su * ld + sv];
    const uint32_t duv = (uint32_t)g.D[(int64_t)su * ld + sv];
    const uint32_t wn = (uint32_t)w;
    int32_t mode = EDGE_NOOP;
    if (wn < w_old) mode = (wn < duv) ? EDGE_DECREASE : EDGE_NOOP;
    else if (wn > w_old) mode = (w_old == duv && duv < INF) ? EDGE_INCREASE : EDGE_NOOP;
    if (lane == 0) {
        Ctl *c = g.ctl;
        c->edge_mode = mode;
        c->w_old = (int32_t)w_old;
        c->duv = (int32_t)duv;
        c->flagged = 0;
        c->rows = 0;
        c->full_scans = 0;
        c->sweeps = 0;
        c->rows_relaxed = 0;
        c->heavy_count = 0;
        c->changed = 0;
        c->rows_changed = 0;
        g.A[(int64_t)su * ld + sv] = w;
        if (g.undirected) g.A[(int64_t)sv * ld + su] = w;
        else g.AT[(int64_t)sv * ld + su] = w;
    }
    wave_list_set_edge(g, sv, su, wn);
    if (g.undirected) wave_list_set_edge(g, su, sv, wn);
}

// The flagged columns of a light row as a set: open addressing over FSET
// slots (at most ROW_CAP keys, so half stay empty and every probe ends),
// key -1 = empty, with each key's position in the row's list.
constexpr int FSET_BITS = 6;
constexpr int FSET = 1 << FSET_BITS;
static_assert(FSET == 64 && 2 * ROW_CAP <= FSET, "one set slot per lane, at most half of them used");
__device__ __forceinline__ uint32_t fset_slot(int32_t x) { return ((uint32_t)x * 0x9E3779B1u) >> (32 - FSET_BITS); }
__device__ __forceinline__ int fset_find(const int32_t *keys, const int32_t *pos, int32_t x) {
    for (uint32_t h = fset_slot(x);; h = (h + 1) & (FSET - 1)) {
        const int32_t key = keys[h];
        if (key == x) return pos[h];
        if (key < 0) return -1;
    }
}

// One light-in-edge pair of a flagged entry e of row i: an edge from an
// unflagged x lowers cm by D[i][x] (+) w, one from a flagged x (its list
// position a) is kept as W[a][e] for the closure; edges at least as heavy
// as best cannot lower the entry and are skipped, and so are those of the
// removed slot.
__device__ __forceinline__ uint32_t light_pull_pair(const int32_t *Drow, int4 p, uint32_t best, uint32_t cm, int e,
                                                    int cnt, int32_t kx, const int32_t *keys, const int32_t *pos,
                                                    uint32_t *W) {
    if ((uint32_t)p.y < best && p.x != kx) {
        const int a = fset_find(keys, pos, p.x);
        if (a >= 0) W[a * cnt + e] = (uint32_t)p.y;
        else cm = min(cm, cat((uint32_t)Drow[p.x], (uint32_t)p.y));
    }
    if ((uint32_t)p.w < best && p.z != kx) {
        const int a = fset_find(keys, pos, p.z);
        if (a >= 0) W[a * cnt + e] = (uint32_t)p.w;
        else cm = min(cm, cat((uint32_t)Drow[p.z], (uint32_t)p.w));
    }
    return cm;
}

// The new entries of a light row (cnt <= ROW_CAP flagged columns list[]),
// one wavefront, every value kept in LDS until the end:
//  1. each flagged entry starts from its best walk whose last edge leaves an
//     unflagged column -- a pull over its light in-edges, lightest eight
//     first, the rest only below the bound they give, stopping at the old
//     value (distances only go up, so an entry back at it is final) -- and
//     the pull keeps the in-edges that come from flagged columns;
//  2. Dijkstra over the flagged columns with those edges closes the set;
//  3. an entry left above its beta_eff could still take an edge missing from
//     the index: a full scan of its column lowers it, and 2-3 repeat until
//     no scan lowers anything.
// Flagged columns are never read from D: their old values may be stale.
// Returns the entry of list position `lane` (INF past cnt).
__device__ inline uint32_t light_row(const DevGraph &g, const FusedArgs &fa, const RowTests &rt, int32_t *Drow,
                                     const int32_t *list, int cnt, int32_t *fsl, int32_t *old, uint32_t *val,
                                     int32_t *keys, int32_t *pos, uint32_t *W, int &sweeps, int &nfs_total) {
    const int lane = lane_id();
    const int g4 = lane >> 2, l4 = lane & 3;
    const int lim = g.lim;
    const int32_t kx = fa.mode == FUSED_REMOVE ? fa.k : -1;
    keys[lane] = -1;
    for (int q = lane; q < cnt * cnt; q += 64) W[q] = INF;
    __threadfence_block();
    int32_t ye = 0;
    uint32_t olde = INF, beta = INF;
    if (lane < cnt) {
        ye = list[lane];
        uint32_t h = fset_slot(ye);
        while (atomicCAS(&keys[h], -1, ye) != -1) h = (h + 1) & (FSET - 1);
        pos[h] = lane;
        olde = flagged_old(fa, rt, ye);
        old[lane] = (int32_t)olde;
        beta = (uint32_t)g.nin_beta[ye];
        if (lim < NIN_L) beta = min(beta, (uint32_t)g.nin[(int64_t)ye * NIN_L + lim].y);
    }
    __threadfence_block();
    for (int e = g4; e < cnt; e += 16) {
        const int32_t y = list[e];
        const uint32_t floor = (uint32_t)old[e];
        const int4 *L4 = reinterpret_cast<const int4 *>(g.nin + (int64_t)y * NIN_L);
        int4 p0 = index_pair(L4, lim, 2 * l4), p1 = index_pair(L4, lim, 8 + 2 * l4);
        int4 p2 = index_pair(L4, lim, 16 + 2 * l4), p3 = index_pair(L4, lim, 24 + 2 * l4);
        uint32_t best = group4_min(light_pull_pair(Drow, p0, INF, INF, e, cnt, kx, keys, pos, W));
        uint32_t wl = (uint32_t)__shfl(p0.w, 3, 4);  // the eighth entry
        for (int c0 = 32; best > floor && wl < best; c0 += 32) {
            uint32_t cm = light_pull_pair(Drow, p1, best, INF, e, cnt, kx, keys, pos, W);
            cm = light_pull_pair(Drow, p2, best, cm, e, cnt, kx, keys, pos, W);
            cm = light_pull_pair(Drow, p3, best, cm, e, cnt, kx, keys, pos, W);
            best = min(best, group4_min(cm));
            wl = (uint32_t)__shfl(p3.w, 3, 4);
            if (c0 >= lim || best <= floor || wl >= best) break;
            p0 = index_pair(L4, lim, c0 + 2 * l4);
            p1 = index_pair(L4, lim, c0 + 8 + 2 * l4);
            p2 = index_pair(L4, lim, c0 + 16 + 2 * l4);
            p3 = index_pair(L4, lim, c0 + 24 + 2 * l4);
            best = min(best, group4_min(light_pull_pair(Drow, p0, best, INF, e, cnt, kx, keys, pos, W)));
            wl = (uint32_t)__shfl(p0.w, 3, 4);
        }
        if (l4 == 0) val[e] = best;
    }
    __threadfence_block();
    ++sweeps;
    // Dijkstra: weights >= 0 and cat is monotone, so the unsettled entry of
    // smallest value is final
    uint32_t dist = lane < cnt ? val[lane] : INF;
    const int32_t *Min = in_matrix(g);
    for (;;) {
        bool done = lane >= cnt;
        for (int it = 0; it < cnt; ++it) {
            const unsigned long long key =
                wave_min_key(done ? ~0ull : (((unsigned long long)dist << 32) | (uint32_t)lane));
            const uint32_t da = (uint32_t)(key >> 32);
            if (key == ~0ull || da >= INF) break;  // wave-uniform
            const int a = (int)(key & 63u);
            if (lane == a) done = true;
            if (!done) dist = min(dist, cat(da, W[a * cnt + lane]));
        }
        // entries that an edge missing from the index could still lower:
        // full scans of their columns against the row as it stands
        unsigned long long need = __ballot(lane < cnt && dist > beta && dist > olde);
        if (!need) break;
        if (lane < cnt) Drow[ye] = (int32_t)dist;
        __threadfence_block();
        nfs_total += __popcll(need);
        bool lowered = false;
        while (need) {
            const int f = __ffsll((long long)need) - 1;
            need &= need - 1;
            const uint32_t df = (uint32_t)__shfl((int)dist, f);
            const uint32_t b = wave_min_plus_below(Drow, Min + (int64_t)list[f] * g.ld, g.n_slots, df);
            if (b < df) {
                lowered = true;
                if (lane == f) {
                    dist = b;
                    Drow[ye] = (int32_t)b;
                }
            }
            __threadfence_block();
        }
        ++sweeps;
        if (!lowered) break;
    }
    return dist;
}


// Per-wavefront LDS of light_row when the caller carves it from one region:
// W (ROW_CAP^2 words), the set's keys and positions, the values, the old
// values and a scratch list.
constexpr int LIGHT_ROW_WORDS = ROW_CAP * ROW_CAP + 2 * FSET + 3 * ROW_CAP;
struct LightRowLds {
    uint32_t *W, *val;
    int32_t *keys, *pos, *old, *fsl;
};
__device__ __forceinline__ LightRowLds light_row_lds(uint32_t *base) {
    LightRowLds l;
    l.W = base;
    l.keys = reinterpret_cast<int32_t *>(base + ROW_CAP * ROW_CAP);
    l.pos = l.keys + FSET;
    l.val = reinterpret_cast<uint32_t *>(l.pos + FSET);
    l.old = reinterpret_cast<int32_t *>(l.val + ROW_CAP);
    l.fsl = l.old + ROW_CAP;
    return l;
}

APSP_SR_END
}  // namespace apsp
