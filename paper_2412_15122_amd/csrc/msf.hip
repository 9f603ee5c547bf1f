// Node removal (and tight edge increase) on an undirected minimax graph by
// its minimum spanning forest: the refined need_update list of Algorithms 11
// and 12 (Theorem 6) computed directly, with work that follows the pairs
// whose distance can change rather than the need_update mask.
//
// With max in place of +, ties are structural (minimax distances of an
// undirected graph form an ultrametric), and the mask of Corollary 3 covers
// most pairs while few of them change.  The forest gives the exact answer:
//   * minimax distances are the largest edge on the path between the two
//     nodes in any minimum spanning forest T of G;
//   * a pair whose T-path avoids k keeps its path in G - k, hence its
//     distance (removing a node never lowers one);
//   * T - k falls into d pieces (the subtrees of k's tree neighbours); a
//     minimum spanning forest of G - k is T - k plus a minimum spanning
//     forest of the pieces joined by the lightest edge between each pair
//     (cycle property: an edge inside a piece closes a cycle of T inside
//     that piece), so for i in piece a and j in piece b the new distance is
//       max(D[i][x_ab], W_ab, D[y_ab][j])
//     where the piece tree's path from a to b leaves a at x_ab, enters b at
//     y_ab, and W_ab is the largest of its edge weights and of the distances
//     inside the pieces it crosses (all unchanged: same-piece pairs keep
//     their T-path).
// A tight increase of edge e = (u, v) is the same argument with one piece
// boundary: T is taken as a forest of the graph before the change (e at its
// old weight).  If e is not in T, T is still a minimum spanning forest after
// the change and no distance moves; otherwise T - e has two pieces, pairs
// inside a piece keep their T-path, and a pair across them takes
// max(D[i][x], W, D[y][j]) with (x, y) the lightest edge that now joins the
// pieces (e at its new weight among the candidates).
// T is built by Boruvka rounds over the light in-edge index (each node's
// lightest edges, ties broken by slot pair), and trusted only with a
// certificate: every edge left out of the index weighs at least its
// endpoint's bound, so the forest is minimum when its heaviest edge in each
// component is no heavier than the bound of every node there, and it spans
// G's components when each component's size equals the number of nodes its
// root reaches in D.  Anything the certificate or a size limit rejects is
// reported, and the caller runs the mask and recompute instead.
#include "apsp_internal.h"
#include "device_common.h"
#include "msf.h"

namespace apsp {

namespace {

constexpr unsigned long long NO_EDGE = ~0ull;

// An edge's key: weight, then the slot pair -- distinct for distinct edges,
// equal from both ends.  Slots fit in 16 bits (MSF_MAX_PITCH).
__device__ __forceinline__ unsigned long long edge_key(uint32_t w, int32_t x, int32_t y) {
    const uint32_t a = (uint32_t)min(x, y), b = (uint32_t)max(x, y);
    return ((unsigned long long)w << 32) | ((unsigned long long)a << 16) | b;
}
__device__ __forceinline__ int32_t key_a(unsigned long long k) { return (int32_t)((k >> 16) & 0xffffu); }
__device__ __forceinline__ int32_t key_b(unsigned long long k) { return (int32_t)(k & 0xffffu); }
__device__ __forceinline__ uint32_t key_w(unsigned long long k) { return (uint32_t)(k >> 32); }

__device__ __forceinline__ unsigned long long wave_min64(unsigned long long v) {
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)v, o);
        const uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)(v >> 32), o);
        const unsigned long long u = ((unsigned long long)hi << 32) | lo;
        v = u < v ? u : v;
    }
    return v;
}

// ---- Boruvka rounds --------------------------------------------------------

__global__ void k_msf_init(DevGraph g, MsfWork w) {
    const int32_t x = blockIdx.x * blockDim.x + threadIdx.x;
    const int n = g.n_slots;
    if (x < g.P) {
        w.label[x] = (x < n && g.id_of_slot[x] >= 0) ? x : -1;
        w.hook[x] = x;
        w.best[x] = NO_EDGE;
        w.comp_max[x] = 0;
        w.comp_size[x] = 0;
        w.pidx[x] = -1;
    }
    if (x < (g.P + 31) / 32) w.rowchg[x] = 0u;
    if (x < MSF_INFO) w.info[x] = 0;
    if (x == 0) w.info[MI_ACTIVE] = 1;
    if (x < MSF_DMAX * MSF_DMAX) w.table[x] = NO_EDGE;
}

// Each live node's lightest index edge to another component, folded into its
// component's best edge (one wavefront per node, one lane per entry).  For a
// raised edge (eu, ev) the forest is the one of the graph before the change:
// the edge also counts at its old weight ew (its index entries, if any, hold
// the new weight, which is heavier and loses).
__global__ __launch_bounds__(256) void k_msf_min(DevGraph g, MsfWork w, int32_t eu, int32_t ev, uint32_t ew) {
    if (!w.info[MI_ACTIVE]) return;
    const int32_t x = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (x >= g.n_slots) return;  // wave-uniform
    const int32_t lx = w.label[x];
    if (lx < 0) return;
    const int lane = lane_id();
    const int cnt = min(g.nin_cnt[x], g.lim);
    unsigned long long key = NO_EDGE;
    if (lane < cnt) {
        const int2 e = g.nin[(int64_t)x * NIN_L + lane];
        const int32_t ly = e.x >= 0 && e.x < g.n_slots ? w.label[e.x] : -1;
        if (ly >= 0 && ly != lx) key = edge_key((uint32_t)e.y, x, e.x);
    }
    if (lane == 0 && (x == eu || x == ev)) {
        const int32_t y = x == eu ? ev : eu;
        const int32_t ly = w.label[y];
        if (ly >= 0 && ly != lx && ew < INF) key = min(key, edge_key(ew, x, y));
    }
    key = wave_min64(key);
    // the best edge only falls: a read at or below the key (stale reads are
    // higher, never lower) makes the atomic useless -- and the nodes of a
    // large component would all queue on its one word
    if (lane == 0 && key != NO_EDGE && key < w.best[lx]) atomicMin(&w.best[lx], key);
}

// Every component root hooks to the component across its best edge and
// records the edge; of two components that pick the same edge, the one with
// the larger root hooks (keys are distinct, so no other cycle forms).
__global__ void k_msf_hook(DevGraph g, MsfWork w) {
    if (!w.info[MI_ACTIVE]) return;
    const int32_t c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= g.n_slots || w.label[c] != c) return;
    const unsigned long long key = w.best[c];
    if (key == NO_EDGE) return;
    const int32_t la = w.label[key_a(key)], lb = w.label[key_b(key)];
    const int32_t o = la == c ? lb : la;
    if (o < 0 || o == c) {
        atomicOr(&w.info[MI_FAIL], MSF_FAIL_STATE);
        return;
    }
    if (w.best[o] == key && c < o) return;  // o hooks to c over this edge
    w.hook[c] = o;
    const int32_t t = atomicAdd(&w.info[MI_TREE], 1);
    if (t < g.P) {
        w.tree_a[t] = key_a(key);
        w.tree_b[t] = key_b(key);
        w.tree_w[t] = (int32_t)key_w(key);
    } else {
        atomicOr(&w.info[MI_FAIL], MSF_FAIL_STATE);
    }
    atomicAdd(&w.info[MI_HOOKS], 1);
}

// Labels follow the hooks to the new roots (bounded walk); best edges reset.
// Thread 0 ends the rounds once a round made no hook.
__global__ void k_msf_relabel(DevGraph g, MsfWork w) {
    if (!w.info[MI_ACTIVE]) return;
    const int32_t x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x == 0) {
        if (w.info[MI_HOOKS] == 0) w.info[MI_ACTIVE] = 0;
        w.info[MI_HOOKS] = 0;
    }
    if (x >= g.n_slots) return;
    w.best[x] = NO_EDGE;
    int32_t r = w.label[x];
    if (r < 0) return;
    for (int s = 0; w.hook[r] != r; ++s) {
        if (s >= MSF_MAX_HOOK_WALK) {
            atomicOr(&w.info[MI_FAIL], MSF_FAIL_DEEP);
            break;
        }
        r = w.hook[r];
    }
    w.label[x] = r;
}

// ---- certificate -----------------------------------------------------------

// Component sizes and heaviest forest edges.  Most slots share one
// component: the lanes of a wavefront that agree with its first valid lane
// combine into one atomic (one counter hit by every slot would serialize),
// the others add their own.
__global__ void k_msf_comp_stats(DevGraph g, MsfWork w) {
    const int32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    const int lane = lane_id();
    const int32_t trees = min(w.info[MI_TREE], g.P);
    // heaviest forest edge per component
    const int32_t le = t < trees ? w.label[w.tree_a[t]] : -1;
    const int32_t we = t < trees ? w.tree_w[t] : 0;
    unsigned long long m = __ballot(le >= 0);
    if (m) {
        const int first = __ffsll((long long)m) - 1;
        const int32_t lf = __shfl(le, first);
        const bool same = le >= 0 && le == lf;
        uint32_t v = same ? (uint32_t)we : 0u;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) v = max(v, (uint32_t)__shfl_xor((int)v, o));
        if (lane == first) atomicMax(&w.comp_max[lf], (int32_t)v);
        if (le >= 0 && !same) atomicMax(&w.comp_max[le], we);
    }
    // size per component
    const int32_t ls = t < g.n_slots ? w.label[t] : -1;
    m = __ballot(ls >= 0);
    if (m) {
        const int first = __ffsll((long long)m) - 1;
        const int32_t lf = __shfl(ls, first);
        const bool same = ls >= 0 && ls == lf;
        const int cnt = __popcll(__ballot(same));
        if (lane == first) atomicAdd(&w.comp_size[lf], cnt);
        if (ls >= 0 && !same) atomicAdd(&w.comp_size[ls], 1);
    }
}

// Per live node: its component's heaviest forest edge is no heavier than the
// node's index bound (every unlisted or unused edge weighs at least it).  Per
// root (one wavefront): the nodes its row of D reaches are its component.
__global__ __launch_bounds__(256) void k_msf_certify(DevGraph g, MsfWork w) {
    const int32_t x = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (x >= g.n_slots) return;  // wave-uniform
    const int32_t lx = w.label[x];
    if (lx < 0) return;
    const int lane = lane_id();
    if (lane == 0) {
        uint32_t beta = (uint32_t)g.nin_beta[x];
        if (g.lim < NIN_L) beta = min(beta, (uint32_t)g.nin[(int64_t)x * NIN_L + g.lim].y);
        if ((uint32_t)w.comp_max[lx] > beta) atomicOr(&w.info[MI_FAIL], MSF_FAIL_CERT);
    }
    if (lx != x) return;
    // the root's row: 16-byte loads, four per lane in flight (rows are padded
    // to a multiple of 128 entries; slots past n_slots are dead)
    const int32_t *Dr = g.D + (int64_t)x * g.ld;
    const int32_t n4 = (g.n_slots + 3) & ~3;
    int reach = 0;
    for (int32_t y0 = lane * 4; y0 < n4; y0 += 64 * 4 * 4) {
        uint4 dv[4], iv[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int32_t y = y0 + q * 256;
            dv[q] = make_uint4(INF, INF, INF, INF);
            iv[q] = make_uint4(0, 0, 0, 0);
            if (y < n4) {
                dv[q] = *reinterpret_cast<const uint4 *>(Dr + y);
                iv[q] = *reinterpret_cast<const uint4 *>(g.id_of_slot + y);
            }
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int32_t y = y0 + q * 256;
            reach += (dv[q].x < INF && (int32_t)iv[q].x >= 0 && y < g.n_slots) +
                     (dv[q].y < INF && (int32_t)iv[q].y >= 0 && y + 1 < g.n_slots) +
                     (dv[q].z < INF && (int32_t)iv[q].z >= 0 && y + 2 < g.n_slots) +
                     (dv[q].w < INF && (int32_t)iv[q].w >= 0 && y + 3 < g.n_slots);
        }
    }
    reach = wave_sum(reach);
    if (lane == 0 && reach != w.comp_size[x]) atomicOr(&w.info[MI_FAIL], MSF_FAIL_SPAN);
}

// ---- pieces of T - k (one work-group, union-find in LDS) --------------------
// For a raised edge (k < 0): the pieces of T - (eu, ev), two when the edge is
// in T, none when it is not (then no distance changes).

__device__ __forceinline__ int32_t uf_find(int32_t *par, int32_t x) {
    int32_t p = par[x];
    while (p != x) {  // path halving: a parent pointer only moves up
        const int32_t gp = par[p];
        if (gp != p) par[x] = gp;
        x = p;
        p = gp;
    }
    return x;
}

__global__ __launch_bounds__(1024) void k_msf_pieces(DevGraph g, MsfWork w, int32_t k, int32_t eu, int32_t ev) {
    extern __shared__ int32_t par[];  // n_slots words
    __shared__ int32_t s_root[MSF_DMAX], s_size[MSF_DMAX];
    __shared__ int32_t s_d, s_fail, s_small, s_comp;
    const int n = g.n_slots;
    const int tid = threadIdx.x;
    const int32_t trees = min(w.info[MI_TREE], g.P);
    for (int32_t x = tid; x < n; x += blockDim.x) par[x] = x;
    if (tid == 0) { s_d = 0; s_fail = 0; s_small = 0; s_comp = 0; }
    if (tid < MSF_DMAX) s_size[tid] = 0;
    __syncthreads();
    for (int32_t e = tid; e < trees; e += blockDim.x) {
        const int32_t a = w.tree_a[e], b = w.tree_b[e];
        if (k >= 0 && (a == k || b == k)) {
            const int32_t slot = atomicAdd(&s_d, 1);
            if (slot < MSF_DMAX) s_root[slot] = a == k ? b : a;
            continue;
        }
        if (k < 0 && ((a == eu && b == ev) || (a == ev && b == eu))) {  // one tree edge at most (distinct keys)
            s_root[0] = eu;
            s_root[1] = ev;
            s_d = 2;
            continue;
        }
        for (int tries = 0;; ++tries) {
            if (tries >= 4096) { atomicOr(&s_fail, MSF_FAIL_STATE); break; }
            int32_t ra = uf_find(par, a), rb = uf_find(par, b);
            if (ra == rb) break;
            if (ra > rb) { const int32_t t = ra; ra = rb; rb = t; }
            if (atomicCAS(&par[rb], rb, ra) == rb) break;  // the larger root under the smaller
        }
    }
    __syncthreads();
    const int d = s_d;
    if (d > MSF_DMAX) {
        if (tid == 0) { w.info[MI_FAIL] |= MSF_FAIL_DEGREE | s_fail; w.info[MI_D] = d; }
        return;
    }
    // the piece of each of k's tree neighbours, then of every node of k's
    // component (other than k)
    __syncthreads();
    if (tid < d) s_root[tid] = uf_find(par, s_root[tid]);
    __syncthreads();
    if (k < 0 && d == 0) {  // a raised edge outside T: nothing changes
        if (tid == 0) {
            w.info[MI_FAIL] |= s_fail;
            w.info[MI_D] = 0;
            w.info[MI_SMALL] = 0;
        }
        return;
    }
    const int32_t lk = w.label[k >= 0 ? k : eu];
    for (int32_t x = tid; x < n; x += blockDim.x) {
        if (x == k || w.label[x] != lk || lk < 0) continue;
        atomicAdd(&s_comp, 1);
        const int32_t r = uf_find(par, x);
        int p = -1;
        for (int q = 0; q < d; ++q)
            if (s_root[q] == r) p = q;
        if (p < 0) { atomicOr(&s_fail, MSF_FAIL_STATE); continue; }
        w.pidx[x] = p;
        atomicAdd(&s_size[p], 1);
    }
    __syncthreads();
    int giant = 0;
    for (int q = 1; q < d; ++q)
        if (s_size[q] > s_size[giant]) giant = q;
    // the nodes of every piece but the largest: the rows the update sweeps
    for (int32_t x = tid; x < n; x += blockDim.x) {
        const int32_t p = w.pidx[x];
        if (p >= 0 && p != giant) w.small[atomicAdd(&s_small, 1)] = x;
    }
    __syncthreads();
    if (tid == 0) {
        w.info[MI_FAIL] |= s_fail;
        w.info[MI_D] = d;
        w.info[MI_SMALL] = s_small;
        w.info[MI_GIANT] = giant;
        w.info[MI_COMP] = s_comp;
    }
    if (tid < d) w.psize[tid] = s_size[tid];
}

// ---- the new distances -----------------------------------------------------

// The lightest edge of G - k from small node x to every other piece (one
// work-group per small node; both directions of the table).
__global__ __launch_bounds__(256) void k_msf_replace(DevGraph g, MsfWork w) {
    __shared__ unsigned long long s_best[MSF_DMAX];
    const int32_t x = w.small[blockIdx.x];
    const int32_t pa = w.pidx[x];
    const int d = w.info[MI_D];
    if (threadIdx.x < MSF_DMAX) s_best[threadIdx.x] = NO_EDGE;
    __syncthreads();
    const int32_t *Ar = g.A + (int64_t)x * g.ld;
    for (int32_t y = threadIdx.x; y < g.n_slots; y += blockDim.x) {
        const int32_t pb = w.pidx[y];
        if (pb < 0 || pb == pa) continue;
        const uint32_t wt = (uint32_t)Ar[y];
        if (wt < INF) atomicMin(&s_best[pb], edge_key(wt, x, y));
    }
    __syncthreads();
    if ((int)threadIdx.x < d && s_best[threadIdx.x] != NO_EDGE) {
        atomicMin(&w.table[pa * MSF_DMAX + threadIdx.x], s_best[threadIdx.x]);
        atomicMin(&w.table[threadIdx.x * MSF_DMAX + pa], s_best[threadIdx.x]);
    }
}

// One work-group: the minimum spanning forest of the d pieces (Prim, one
// thread), then, from every piece a (one thread each), a walk of that forest
// recording for each piece b reached the exit node x_ab in a, the entry node
// y_ab in b, and W_ab (the largest edge weight and in-piece distance along
// the way); W_ab = INF for pieces not reached.
__global__ __launch_bounds__(64) void k_msf_pairs(DevGraph g, MsfWork w) {
    __shared__ int32_t s_par[MSF_DMAX];
    __shared__ unsigned long long s_edge[MSF_DMAX];
    __shared__ int32_t s_stack[MSF_DMAX][MSF_DMAX];  // per source: pieces to visit
    const int d = w.info[MI_D];
    const int a = threadIdx.x;
    if (a == 0) {
        unsigned long long dist[MSF_DMAX];
        bool in_tree[MSF_DMAX];
        for (int q = 0; q < d; ++q) {
            s_par[q] = -1;
            s_edge[q] = NO_EDGE;
            dist[q] = NO_EDGE;
            in_tree[q] = false;
        }
        for (int it = 0; it < d; ++it) {
            int best = -1;
            for (int q = 0; q < d; ++q)
                if (!in_tree[q] && (best < 0 || dist[q] < dist[best])) best = q;
            in_tree[best] = true;  // a new tree starts where dist is NO_EDGE
            for (int q = 0; q < d; ++q) {
                const unsigned long long e = w.table[best * MSF_DMAX + q];
                if (!in_tree[q] && e < dist[q]) {
                    dist[q] = e;
                    s_par[q] = best;
                    s_edge[q] = e;
                }
            }
        }
    }
    __syncthreads();
    if (a >= d) return;
    // (piece, entry node, W, exit node of a) per visit; the forest has at most
    // d - 1 edges, so a piece is pushed once
    int32_t top = 0;
    int32_t *stk = s_stack[a];
    for (int b = 0; b < d; ++b) {
        w.wab[a * MSF_DMAX + b] = (int32_t)INF;
        w.xab[a * MSF_DMAX + b] = -1;
        w.yab[a * MSF_DMAX + b] = -1;
    }
    unsigned long long seen = 1ull << a;
    stk[top++] = a;
    while (top > 0) {
        const int c = stk[--top];
        const int32_t yin = c == a ? -1 : w.yab[a * MSF_DMAX + c];
        const uint32_t Wc = c == a ? 0u : (uint32_t)w.wab[a * MSF_DMAX + c];
        const int32_t xfirst = c == a ? -1 : w.xab[a * MSF_DMAX + c];
        for (int q = 0; q < d; ++q) {
            // forest edges of c: to its parent, and from its children
            unsigned long long e = NO_EDGE;
            if (s_par[c] == q) e = s_edge[c];
            else if (s_par[q] == c) e = s_edge[q];
            if (e == NO_EDGE || ((seen >> q) & 1ull)) continue;
            seen |= 1ull << q;
            const int32_t ea = key_a(e), eb = key_b(e);
            const int32_t p = w.pidx[ea] == c ? ea : eb;   // the edge's end in c
            const int32_t r = p == ea ? eb : ea;            // and in q
            uint32_t Wq = max(Wc, key_w(e));
            if (c != a) Wq = max(Wq, (uint32_t)g.D[(int64_t)yin * g.ld + p]);
            w.wab[a * MSF_DMAX + q] = (int32_t)Wq;
            w.xab[a * MSF_DMAX + q] = c == a ? p : xfirst;
            w.yab[a * MSF_DMAX + q] = r;
            stk[top++] = q;
        }
    }
}

// Row x of every small piece (one work-group per node): each entry of x to
// another piece takes its new value; the entries to the giant piece are
// written to its rows as well (D is symmetric).  Changed entries are counted
// (both orders) and their rows marked.
__global__ __launch_bounds__(256) void k_msf_apply(DevGraph g, MsfWork w) {
    __shared__ uint32_t s_dx[MSF_DMAX], s_w[MSF_DMAX];
    __shared__ int32_t s_y[MSF_DMAX];
    __shared__ unsigned long long s_changed;
    const int32_t x = w.small[blockIdx.x];
    const int32_t pa = w.pidx[x];
    const int d = w.info[MI_D], giant = w.info[MI_GIANT];
    const int32_t *Dx = g.D + (int64_t)x * g.ld;
    if (threadIdx.x < d) {
        const int b = threadIdx.x;
        const int32_t xab = w.xab[pa * MSF_DMAX + b];
        s_w[b] = (uint32_t)w.wab[pa * MSF_DMAX + b];
        s_y[b] = w.yab[pa * MSF_DMAX + b];
        s_dx[b] = xab >= 0 ? (uint32_t)Dx[xab] : INF;
    }
    if (threadIdx.x == 0) s_changed = 0;
    __syncthreads();
    int32_t *Dxw = g.D + (int64_t)x * g.ld;
    unsigned long long mine = 0;
    bool row_changed = false;
    for (int32_t j = threadIdx.x; j < g.n_slots; j += blockDim.x) {
        const int32_t pb = w.pidx[j];
        if (pb < 0 || pb == pa) continue;
        const uint32_t W = s_w[pb];
        const uint32_t v = W >= INF ? INF : max(max(s_dx[pb], W), (uint32_t)g.D[(int64_t)s_y[pb] * g.ld + j]);
        const uint32_t old = (uint32_t)Dxw[j];
        if (v == old) continue;
        Dxw[j] = (int32_t)v;
        ++mine;
        row_changed = true;
        if (pb == giant) {  // the mirrored entry: row j is swept by no work-group
            g.D[(int64_t)j * g.ld + x] = (int32_t)v;
            ++mine;
            atomicOr(&w.rowchg[j >> 5], 1u << (j & 31));
        }
    }
    if (mine) atomicAdd(&s_changed, mine);
    if (__any(row_changed) && lane_id() == 0) atomicOr(&w.rowchg[x >> 5], 1u << (x & 31));
    __syncthreads();
    if (threadIdx.x == 0 && s_changed) atomicAdd(&g.ctl->changed, s_changed);
}

// Phi' (rows with a changed entry) into the control block.
__global__ __launch_bounds__(256) void k_msf_finish(DevGraph g, MsfWork w) {
    __shared__ uint32_t red[8];
    int c = 0;
    for (int32_t q = threadIdx.x; q < (g.n_slots + 31) / 32; q += blockDim.x) c += __popc(w.rowchg[q]);
    c = block_sum256(c, red);
    if (threadIdx.x == 0) g.ctl->rows_changed += c;
}

}  // namespace

MsfWork msf_work(int32_t *scratch, int32_t P) {
    MsfWork w{};
    int64_t off = 0;
    auto take = [&](int64_t ints) {
        int32_t *p = scratch + off;
        off += (ints + 63) & ~63ll;
        return p;
    };
    w.label = take(P);
    w.hook = take(P);
    w.best = reinterpret_cast<unsigned long long *>(take(2 * (int64_t)P));
    w.tree_a = take(P);
    w.tree_b = take(P);
    w.tree_w = take(P);
    w.comp_max = take(P);
    w.comp_size = take(P);
    w.pidx = take(P);
    w.small = take(P);
    w.rowchg = reinterpret_cast<uint32_t *>(take((P + 31) / 32));
    w.info = take(MSF_INFO);
    w.psize = take(MSF_DMAX);
    w.table = reinterpret_cast<unsigned long long *>(take(2 * MSF_DMAX * MSF_DMAX));
    w.xab = take(MSF_DMAX * MSF_DMAX);
    w.yab = take(MSF_DMAX * MSF_DMAX);
    w.wab = take(MSF_DMAX * MSF_DMAX);
    w.ints = off;
    return w;
}

hipError_t msf_configure() {
    static hipError_t status = hipErrorNotReady;
    if (status == hipErrorNotReady)
        status = hipFuncSetAttribute((const void *)k_msf_pieces, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     MSF_MAX_PITCH * (int)sizeof(int32_t));
    return status;
}

void launch_msf_forest(const DevGraph &g, const MsfWork &w, int32_t k, int32_t eu, int32_t ev, int32_t ew,
                       int32_t rounds, hipStream_t s) {
    const int32_t n = g.n_slots;
    const int32_t init = std::max<int32_t>(g.P, MSF_DMAX * MSF_DMAX);
    k_msf_init<<<(init + 255) / 256, 256, 0, s>>>(g, w);
    for (int32_t r = 0; r < rounds; ++r) {
        k_msf_min<<<(n + 3) / 4, 256, 0, s>>>(g, w, eu, ev, (uint32_t)ew);
        k_msf_hook<<<(n + 255) / 256, 256, 0, s>>>(g, w);
        k_msf_relabel<<<(n + 255) / 256, 256, 0, s>>>(g, w);
    }
    k_msf_comp_stats<<<(g.P + 255) / 256, 256, 0, s>>>(g, w);
    k_msf_certify<<<(n + 3) / 4, 256, 0, s>>>(g, w);
    k_msf_pieces<<<1, 1024, (size_t)n * sizeof(int32_t), s>>>(g, w, k, eu, ev);
}

void launch_msf_update(const DevGraph &g, const MsfWork &w, int32_t small_count, hipStream_t s) {
    if (small_count > 0) k_msf_replace<<<small_count, 256, 0, s>>>(g, w);
    k_msf_pairs<<<1, 64, 0, s>>>(g, w);
    if (small_count > 0) k_msf_apply<<<small_count, 256, 0, s>>>(g, w);
    k_msf_finish<<<1, 256, 0, s>>>(g, w);
}

}  // namespace apsp
