/*
 * The paper's own warm-start procedures on the CPU -- TEST AND BENCHMARK
 * INFRASTRUCTURE ONLY (used by tests/ and the benchmark's CPU baseline leg;
 * nothing on the GPU path calls it).  It shares no code with the HIP
 * library.
 *
 * One thread, plain loops, the steps in the paper's order, so that measured
 * warm/cold time ratios can be set beside the paper's Tables 1-4:
 *
 *   pc_fw             the cold start: textbook Floyd-Warshall (Section 1).
 *   pc_remove         Algorithm 5: need_update_list by Corollary 3,
 *                     Cost (Definition 1), Floyd-Warshall on
 *                     G - G_k when Cost > delta, else copy M_G and run one
 *                     dense Dijkstra on G - G_k from every row with a
 *                     non-empty list, stopping once the row's listed nodes
 *                     are settled, and take the listed entries.
 *   pc_remove_key     Algorithm 11: a flagged pair stays listed only when k
 *                     is in its key_node_list, built as Algorithm 10 does:
 *                     Algorithm 7's candidates, a Dijkstra path Psi on the
 *                     small graph, then one path through every candidate
 *                     off Psi (Algorithm 8 with Psi in place of {i, j}),
 *                     intersected; then Algorithm 5 from its Cost step.
 *   pc_edge           Algorithm 6: the endpoint whose removal costs less is
 *                     removed (Algorithm 5), then added back with the new
 *                     weight by the add-node theorems of Section 3.1
 *                     (Theorems 1, 2 and 3).
 *   pc_query          Algorithm 7: candidates, small graph, Dijkstra on it.
 *   pc_dijkstra_path  the cold single-pair query (Dijkstra on G).
 *   pc_remove_sample  a bounded timing sample of Algorithm 5 (benchmark).
 *
 * Distances are uint32 with INF = 2^30 (absent edge / unreachable) and
 * saturating sums.  Matrices are row-major n x n int32; results of a removal
 * are (n-1) x (n-1) in the order of the remaining nodes.  `st` receives
 * (Phi, listed pairs, fell back to Floyd-Warshall, Dijkstra runs, and --
 * pc_remove_key -- the pairs Corollary 3 flagged, or -- pc_edge --
 * the removed endpoint): 5 entries.  Every routine returns 0, or -1 when it
 * cannot allocate its work space.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>

#define PC_INF (1u << 30)

static inline uint32_t cat(uint32_t a, uint32_t b) {
    const uint32_t s = a + b;  /* a, b <= 2^30: no wrap */
    return s < PC_INF ? s : PC_INF;
}

/* ---- cold start --------------------------------------------------------- */

static void fw_inplace(int32_t m, uint32_t *D) {
    for (int32_t k = 0; k < m; ++k) {
        const uint32_t *rk = D + (size_t)k * m;
        for (int32_t i = 0; i < m; ++i) {
            uint32_t *ri = D + (size_t)i * m;
            const uint32_t dik = ri[k];
            if (dik >= PC_INF) continue;
            for (int32_t j = 0; j < m; ++j) {
                const uint32_t v = dik + rk[j];
                if (v < ri[j]) ri[j] = v;
            }
        }
    }
}

int pc_fw(int32_t n, const int32_t *A, int32_t *D) {
    memcpy(D, A, (size_t)n * n * sizeof(int32_t));
    for (int32_t i = 0; i < n; ++i) D[(size_t)i * n + i] = 0;
    fw_inplace(n, (uint32_t *)D);
    return 0;
}

/* ---- dense Dijkstra ----------------------------------------------------- */

/* From src over the m x m matrix W (rev: over its transpose, i.e. distances
 * to src).  Nodes with skip[v] set are absent.  With need != NULL it stops
 * once the need_cnt nodes flagged there are settled. */
static void dijkstra(int32_t m, const uint32_t *W, int rev, int32_t src, const uint8_t *skip, uint32_t *dist,
                     int32_t *pred, uint8_t *done, const uint8_t *need, int32_t need_cnt) {
    for (int32_t v = 0; v < m; ++v) {
        dist[v] = PC_INF;
        pred[v] = -1;
        done[v] = skip ? skip[v] : 0;
    }
    dist[src] = 0;
    int32_t left = need_cnt;
    for (int32_t it = 0; it < m; ++it) {
        int32_t u = -1;
        uint32_t best = PC_INF;
        for (int32_t v = 0; v < m; ++v)
            if (!done[v] && dist[v] < best) { best = dist[v]; u = v; }
        if (u < 0) break;
        done[u] = 1;
        if (need && need[u] && --left == 0) break;
        for (int32_t v = 0; v < m; ++v) {
            if (done[v]) continue;
            const uint32_t w = rev ? W[(size_t)v * m + u] : W[(size_t)u * m + v];
            if (w >= PC_INF) continue;
            const uint32_t nd = best + w;
            if (nd < dist[v]) { dist[v] = nd; pred[v] = u; }
        }
    }
}

/* ---- node removal (Algorithms 5 and 11) --------------------------------- */

/* Steps of Algorithm 5 from the Cost test on, given the need_update_list
 * (need[i*n + j]) and its row counts.  Writes the (n-1)^2 result. */
static int remove_from_lists(int32_t n, const uint32_t *A, const uint32_t *D, int32_t k, double delta,
                             const uint8_t *need, const int32_t *cnt, int32_t *D2, int64_t *st, double *cost) {
    const int32_t m = n - 1;
    int64_t phi = 0, listed = 0;
    for (int32_t i = 0; i < n; ++i) {
        phi += cnt[i] > 0;
        listed += cnt[i];
    }
    const double c = n > 1 ? (double)phi / (double)(n - 1) : 0.0;
    if (cost) *cost = c;
    st[0] = phi;
    st[1] = listed;
    st[2] = 0;
    st[3] = 0;
    if (c > delta) {  /* cold start on G - G_k */
        for (int32_t r = 0, i = 0; i < n; ++i) {
            if (i == k) continue;
            for (int32_t s = 0, j = 0; j < n; ++j) {
                if (j == k) continue;
                D2[(size_t)r * m + s++] = (int32_t)(i == j ? 0 : A[(size_t)i * n + j]);
            }
            ++r;
        }
        fw_inplace(m, (uint32_t *)D2);
        st[2] = 1;
        return 0;
    }
    for (int32_t r = 0, i = 0; i < n; ++i) {  /* copy(M_G) without k */
        if (i == k) continue;
        for (int32_t s = 0, j = 0; j < n; ++j) {
            if (j == k) continue;
            D2[(size_t)r * m + s++] = (int32_t)D[(size_t)i * n + j];
        }
        ++r;
    }
    uint32_t *dist = malloc((size_t)n * 4);
    int32_t *pred = malloc((size_t)n * 4);
    uint8_t *done = malloc((size_t)n), *skip = calloc((size_t)n, 1);
    if (!dist || !pred || !done || !skip) {
        free(dist); free(pred); free(done); free(skip);
        return -1;
    }
    skip[k] = 1;
    for (int32_t r = 0, i = 0; i < n; ++i) {
        if (i == k) continue;
        if (cnt[i] > 0) {
            const uint8_t *ni = need + (size_t)i * n;
            dijkstra(n, A, 0, i, skip, dist, pred, done, ni, cnt[i]);
            ++st[3];
            for (int32_t s = 0, j = 0; j < n; ++j) {
                if (j == k) continue;
                if (ni[j]) D2[(size_t)r * m + s] = (int32_t)dist[j];
                ++s;
            }
        }
        ++r;
    }
    free(dist); free(pred); free(done); free(skip);
    return 0;
}

/* need_update_list of removing k: D[i][k] + D[k][j] == D[i][j] < INF. */
static void need_lists(int32_t n, const uint32_t *D, int32_t k, uint8_t *need, int32_t *cnt) {
    const uint32_t *rk = D + (size_t)k * n;
    for (int32_t i = 0; i < n; ++i) {
        uint8_t *ni = need + (size_t)i * n;
        const uint32_t *ri = D + (size_t)i * n;
        const uint32_t dik = ri[k];
        int32_t c = 0;
        for (int32_t j = 0; j < n; ++j) {
            const uint8_t f = i != k && j != k && i != j && ri[j] < PC_INF && cat(dik, rk[j]) == ri[j];
            ni[j] = f;
            c += f;
        }
        cnt[i] = c;
    }
}

int pc_remove(int32_t n, const int32_t *A, const int32_t *D, int32_t k, double delta, int32_t *D2, int64_t *st,
              double *cost) {
    uint8_t *need = malloc((size_t)n * n);
    int32_t *cnt = malloc((size_t)n * 4);
    if (!need || !cnt) { free(need); free(cnt); return -1; }
    need_lists(n, (const uint32_t *)D, k, need, cnt);
    const int rc = remove_from_lists(n, (const uint32_t *)A, (const uint32_t *)D, k, delta, need, cnt, D2, st, cost);
    free(need);
    free(cnt);
    return rc;
}

static int64_t now_ns(void) {
    struct timespec ts;
    clock_gettime(CLOCK_MONOTONIC, &ts);
    return (int64_t)ts.tv_sec * 1000000000 + ts.tv_nsec;
}

/* A bounded timing sample of Algorithm 5 on a graph too large to run it
 * whole on one thread: the need_update_list step in full, then the first
 * max_runs of its Dijkstra runs (rows in order).  No matrix is written.
 * st: Phi, listed pairs, runs timed, ns in the list step, ns in the runs. */
int pc_remove_sample(int32_t n, const int32_t *A, const int32_t *D, int32_t k, int32_t max_runs, int64_t *st) {
    uint8_t *need = malloc((size_t)n * n);
    int32_t *cnt = malloc((size_t)n * 4), *pred = malloc((size_t)n * 4);
    uint32_t *dist = malloc((size_t)n * 4);
    uint8_t *done = malloc((size_t)n), *skip = calloc((size_t)n, 1);
    if (!need || !cnt || !pred || !dist || !done || !skip) {
        free(need); free(cnt); free(pred); free(dist); free(done); free(skip);
        return -1;
    }
    int64_t t0 = now_ns();
    need_lists(n, (const uint32_t *)D, k, need, cnt);
    int64_t phi = 0, listed = 0;
    for (int32_t i = 0; i < n; ++i) {
        phi += cnt[i] > 0;
        listed += cnt[i];
    }
    const int64_t t1 = now_ns();
    skip[k] = 1;
    int32_t runs = 0;
    for (int32_t i = 0; i < n && runs < max_runs; ++i) {
        if (i == k || !cnt[i]) continue;
        dijkstra(n, (const uint32_t *)A, 0, i, skip, dist, pred, done, need + (size_t)i * n, cnt[i]);
        ++runs;
    }
    const int64_t t2 = now_ns();
    st[0] = phi;
    st[1] = listed;
    st[2] = runs;
    st[3] = t1 - t0;
    st[4] = t2 - t1;
    free(need); free(cnt); free(pred); free(dist); free(done); free(skip);
    return 0;
}

/* Key-node work space for one pair. */
typedef struct {
    int32_t *cand, *pred, *succ, *hits, *stamp;
    uint32_t *S, *dist;
    uint8_t *done, *on_psi;
    int32_t cap;
} KeyWork;

static int key_work_init(KeyWork *w, int32_t n) {
    memset(w, 0, sizeof(*w));
    w->cap = n;
    w->cand = malloc((size_t)n * 4);
    w->pred = malloc((size_t)n * 4);
    w->succ = malloc((size_t)n * 4);
    w->hits = malloc((size_t)n * 4);
    w->stamp = malloc((size_t)n * 4);
    w->dist = malloc((size_t)n * 4);
    w->done = malloc((size_t)n);
    w->on_psi = malloc((size_t)n);
    w->S = NULL;
    return w->cand && w->pred && w->succ && w->hits && w->stamp && w->dist && w->done && w->on_psi ? 0 : -1;
}

static void key_work_free(KeyWork *w) {
    free(w->cand); free(w->pred); free(w->succ); free(w->hits); free(w->stamp);
    free(w->dist); free(w->done); free(w->on_psi); free(w->S);
}

/* Is k in the key_node_list of (i, j)?  The list is the intersection of
 * Psi and of one path i -> t -> j for every candidate t off Psi (shortest
 * paths on the small graph: the Dijkstra tree from i and the reverse tree
 * into j), with i and j taken out. */
static int k_is_key(int32_t n, const uint32_t *A, const uint32_t *D, int32_t i, int32_t j, int32_t k, KeyWork *w) {
    const uint32_t dij = D[(size_t)i * n + j];
    int32_t K = 0, ci = -1, cj = -1, ck = -1;
    for (int32_t t = 0; t < n; ++t) {
        if (cat(D[(size_t)i * n + t], D[(size_t)t * n + j]) != dij) continue;
        if (t == i) ci = K;
        if (t == j) cj = K;
        if (t == k) ck = K;
        w->cand[K++] = t;
    }
    if (ci < 0 || cj < 0 || ck < 0) return 0;
    uint32_t *S = realloc(w->S, (size_t)K * K * 4);
    if (!S) return 1;  /* cannot tell: keep the pair listed */
    w->S = S;
    for (int32_t a = 0; a < K; ++a)
        for (int32_t b = 0; b < K; ++b) S[(size_t)a * K + b] = A[(size_t)w->cand[a] * n + w->cand[b]];
    dijkstra(K, S, 0, ci, NULL, w->dist, w->pred, w->done, NULL, 0);
    dijkstra(K, S, 1, cj, NULL, w->dist, w->succ, w->done, NULL, 0);
    /* hits[c]: paths through c, each path counted once per node (stamp:
     * the last path that counted it; with zero-weight edges the two halves
     * of a path may share nodes) */
    memset(w->hits, 0, (size_t)K * 4);
    memset(w->on_psi, 0, (size_t)K);
    for (int32_t c = 0; c < K; ++c) w->stamp[c] = -1;
#define PC_HIT(c, p) do { if (w->stamp[c] != (p)) { w->stamp[c] = (p); ++w->hits[c]; } } while (0)
    int32_t paths = 1;
    for (int32_t c = cj; c >= 0; c = w->pred[c]) {  /* Psi */
        w->on_psi[c] = 1;
        PC_HIT(c, 0);
        if (c == ci) break;
    }
    for (int32_t t = 0; t < K; ++t) {
        if (w->on_psi[t]) continue;
        const int32_t p = paths++;
        for (int32_t c = t; c >= 0 && c != ci; c = w->pred[c]) PC_HIT(c, p);  /* i -> t */
        PC_HIT(ci, p);
        for (int32_t c = w->succ[t]; c >= 0 && c != cj; c = w->succ[c]) PC_HIT(c, p);  /* t -> j */
        PC_HIT(cj, p);
    }
#undef PC_HIT
    return w->hits[ck] == paths;
}

int pc_remove_key(int32_t n, const int32_t *A, const int32_t *D, int32_t k, double delta, int32_t *D2, int64_t *st,
                  double *cost) {
    uint8_t *need = malloc((size_t)n * n);
    int32_t *cnt = malloc((size_t)n * 4);
    KeyWork w;
    if (!need || !cnt || key_work_init(&w, n)) {
        free(need); free(cnt); key_work_free(&w);
        return -1;
    }
    need_lists(n, (const uint32_t *)D, k, need, cnt);  /* the pairs Corollary 3 flags */
    int64_t flagged = 0;
    for (int32_t i = 0; i < n; ++i) {
        if (!cnt[i]) continue;
        uint8_t *ni = need + (size_t)i * n;
        for (int32_t j = 0; j < n; ++j) {
            if (!ni[j]) continue;
            ++flagged;
            if (!k_is_key(n, (const uint32_t *)A, (const uint32_t *)D, i, j, k, &w)) {
                ni[j] = 0;
                --cnt[i];
            }
        }
    }
    const int rc = remove_from_lists(n, (const uint32_t *)A, (const uint32_t *)D, k, delta, need, cnt, D2, st, cost);
    st[4] = flagged;
    key_work_free(&w);
    free(need);
    free(cnt);
    return rc;
}

/* ---- edge change (Algorithm 6) ------------------------------------------ */

int pc_edge(int32_t n, const int32_t *A, const int32_t *D, int32_t undirected, int32_t u, int32_t v, int32_t w,
            double delta, int32_t *Dout, int64_t *st) {
    const uint32_t *Du = (const uint32_t *)D;
    const int32_t m = n - 1;
    uint8_t *need = malloc((size_t)n * n);
    int32_t *cnt = malloc((size_t)n * 4), *D2 = malloc((size_t)m * m * 4);
    uint32_t *Ap = malloc((size_t)n * n * 4), *out = malloc((size_t)n * 4), *in = malloc((size_t)n * 4);
    if (!need || !cnt || !D2 || !Ap || !out || !in) {
        free(need); free(cnt); free(D2); free(Ap); free(out); free(in);
        return -1;
    }
    /* Cost of removing each endpoint; the cheaper one goes. */
    double cost_u, cost_v;
    int64_t phi;
    need_lists(n, Du, u, need, cnt);
    phi = 0;
    for (int32_t i = 0; i < n; ++i) phi += cnt[i] > 0;
    cost_u = (double)phi / (double)(n - 1);
    need_lists(n, Du, v, need, cnt);
    phi = 0;
    for (int32_t i = 0; i < n; ++i) phi += cnt[i] > 0;
    cost_v = (double)phi / (double)(n - 1);
    const int32_t k = cost_u < cost_v ? u : v;
    if (k == u) need_lists(n, Du, u, need, cnt);
    int rc = remove_from_lists(n, (const uint32_t *)A, Du, k, delta, need, cnt, D2, st, NULL);
    st[4] = k;
    if (rc) goto done;
    /* G': the edge re-weighted; k added back (Section 3.1). */
    memcpy(Ap, A, (size_t)n * n * 4);
    Ap[(size_t)u * n + v] = (uint32_t)w;
    if (undirected) Ap[(size_t)v * n + u] = (uint32_t)w;
    /* out[c] = min_t w(k, t) + D[t][c]; in[r] = min_t D[r][t] + w(t, k) (compact r, c, t) */
    for (int32_t c = 0; c < m; ++c) out[c] = PC_INF;
    for (int32_t r = 0; r < m; ++r) in[r] = PC_INF;
    for (int32_t t = 0, ot = 0; ot < n; ++ot) {
        if (ot == k) continue;
        const uint32_t wk = Ap[(size_t)k * n + ot];
        if (wk < PC_INF) {
            const uint32_t *rt = (const uint32_t *)D2 + (size_t)t * m;
            for (int32_t c = 0; c < m; ++c) {
                const uint32_t x = cat(wk, rt[c]);
                if (x < out[c]) out[c] = x;
            }
        }
        ++t;
    }
    for (int32_t r = 0; r < m; ++r) {
        const uint32_t *rr = (const uint32_t *)D2 + (size_t)r * m;
        uint32_t best = PC_INF;
        for (int32_t t = 0, ot = 0; ot < n; ++ot) {
            if (ot == k) continue;
            const uint32_t x = cat(rr[t], Ap[(size_t)ot * n + k]);
            if (x < best) best = x;
            ++t;
        }
        in[r] = best;
    }
    for (int32_t r = 0, i = 0; i < n; ++i) {
        uint32_t *ro = (uint32_t *)Dout + (size_t)i * n;
        if (i == k) {
            for (int32_t c = 0, j = 0; j < n; ++j) ro[j] = j == k ? 0 : out[c++];
            continue;
        }
        const uint32_t *rr = (const uint32_t *)D2 + (size_t)r * m;
        for (int32_t c = 0, j = 0; j < n; ++j) {
            if (j == k) { ro[j] = in[r]; continue; }
            const uint32_t x = cat(in[r], out[c]);
            ro[j] = x < rr[c] ? x : rr[c];
            ++c;
        }
        ++r;
    }
done:
    free(need); free(cnt); free(D2); free(Ap); free(out); free(in);
    return rc;
}

/* ---- single-pair query (Algorithm 7) ------------------------------------ */

int pc_query(int32_t n, const int32_t *A, const int32_t *D, int32_t i, int32_t j, int32_t *path, int32_t *len,
             int32_t *dist_out) {
    const uint32_t *Au = (const uint32_t *)A, *Du = (const uint32_t *)D;
    const uint32_t dij = Du[(size_t)i * n + j];
    *len = 0;
    *dist_out = (int32_t)dij;
    if (i == j) { path[0] = i; *len = 1; return 0; }
    if (dij >= PC_INF) return 0;
    int32_t *cand = malloc((size_t)n * 4);
    if (!cand) return -1;
    int32_t K = 0, ci = -1, cj = -1;
    for (int32_t t = 0; t < n; ++t) {
        if (cat(Du[(size_t)i * n + t], Du[(size_t)t * n + j]) != dij) continue;
        if (t == i) ci = K;
        if (t == j) cj = K;
        cand[K++] = t;
    }
    uint32_t *S = malloc((size_t)K * K * 4), *dist = malloc((size_t)K * 4);
    int32_t *pred = malloc((size_t)K * 4);
    uint8_t *done = malloc((size_t)K), *need = calloc((size_t)K, 1);
    if (!S || !dist || !pred || !done || !need) {
        free(cand); free(S); free(dist); free(pred); free(done); free(need);
        return -1;
    }
    for (int32_t a = 0; a < K; ++a)
        for (int32_t b = 0; b < K; ++b) S[(size_t)a * K + b] = Au[(size_t)cand[a] * n + cand[b]];
    need[cj] = 1;
    dijkstra(K, S, 0, ci, NULL, dist, pred, done, need, 1);
    int32_t L = 0;
    for (int32_t c = cj; c >= 0; c = pred[c]) {
        path[L++] = cand[c];
        if (c == ci) break;
    }
    for (int32_t a = 0, b = L - 1; a < b; ++a, --b) {
        const int32_t x = path[a]; path[a] = path[b]; path[b] = x;
    }
    *len = L;
    free(cand); free(S); free(dist); free(pred); free(done); free(need);
    return 0;
}

int pc_dijkstra_path(int32_t n, const int32_t *A, int32_t i, int32_t j, int32_t *path, int32_t *len,
                     int32_t *dist_out) {
    uint32_t *dist = malloc((size_t)n * 4);
    int32_t *pred = malloc((size_t)n * 4);
    uint8_t *done = malloc((size_t)n), *need = calloc((size_t)n, 1);
    if (!dist || !pred || !done || !need) {
        free(dist); free(pred); free(done); free(need);
        return -1;
    }
    need[j] = 1;
    dijkstra(n, (const uint32_t *)A, 0, i, NULL, dist, pred, done, need, 1);
    *dist_out = (int32_t)dist[j];
    int32_t L = 0;
    if (dist[j] < PC_INF) {
        for (int32_t c = j; c >= 0; c = pred[c]) path[L++] = c;
        for (int32_t a = 0, b = L - 1; a < b; ++a, --b) {
            const int32_t x = path[a]; path[a] = path[b]; path[b] = x;
        }
    }
    *len = L;
    free(dist); free(pred); free(done); free(need);
    return 0;
}
