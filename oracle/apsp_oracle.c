/*
 * CPU oracle for warm-start all-pairs shortest paths -- TEST INFRASTRUCTURE.
 *
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * may load this library.  The product (the HIP library) never does, and the
 * two share no code, headers or tables.
 *
 * What it computes is the plain definition the warm-start method must reach
 * exactly (paper, Section 1: the shortest-path problem and APSP; notation
 * table: SPD(i,j|G) with SPD(i,i) = 0 and the APSP matrix M_G): the cold APSP
 * matrix of the graph, by two textbook routines the paper names as the cold
 * baselines (Section 1 and Section 3.1: Floyd-Warshall and Dijkstra):
 *
 *   oracle_fw_init / oracle_fw_pivots   Floyd-Warshall, k outermost
 *   oracle_dijkstra_rows                dense O(n^2) Dijkstra per source
 *
 * Arithmetic: weights and distances are int32 in [0, INF] with INF = 2^30
 * meaning "no edge / unreachable".  Path concatenation is the saturating sum
 * a (+) b = min(a + b, INF), evaluated in uint32 so that INF + INF (2^31)
 * cannot overflow.  Matrices are dense, row-major, n x n, no padding.
 *
 * Threads: the pivot loop parallelises over rows i for each k (OpenMP);
 * nthreads <= 0 means the OpenMP default.  Results do not depend on the
 * thread count (integer min is exact and order-free).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_INF 1073741824u

static inline uint32_t oplus(uint32_t a, uint32_t b)
{
    uint32_t s = a + b;
    return s < ORACLE_INF ? s : ORACLE_INF;
}

static void set_threads(int nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
}

int oracle_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* D := A with a zero diagonal (SPD(i,i) = 0).  Returns 0, or -1 on bad input. */
int oracle_fw_init(int32_t n, const int32_t *A, int32_t *D)
{
    if (n < 0 || (n > 0 && (!A || !D))) return -1;
    for (int64_t x = 0; x < (int64_t)n * n; ++x) {
        if (A[x] < 0 || (uint32_t)A[x] > ORACLE_INF) return -1;
    }
    memcpy(D, A, sizeof(int32_t) * (size_t)n * (size_t)n);
    for (int32_t i = 0; i < n; ++i) D[(int64_t)i * n + i] = 0;
    return 0;
}

/*
 * Floyd-Warshall pivots k0 .. k1-1 applied in place:
 *   for k: for i: for j: D[i][j] = min(D[i][j], D[i][k] (+) D[k][j]).
 * oracle_fw_init followed by pivots [0, n) is the full textbook algorithm.
 * Row k is not modified during pivot k (D[k][k] = 0), so rows may be
 * processed in parallel.
 */
int oracle_fw_pivots(int32_t n, int32_t *D, int32_t k0, int32_t k1, int nthreads)
{
    if (n < 0 || k0 < 0 || k1 > n || k0 > k1) return -1;
    set_threads(nthreads);
    uint32_t *M = (uint32_t *)D;
    for (int32_t k = k0; k < k1; ++k) {
        const uint32_t *rowk = M + (int64_t)k * n;
#pragma omp parallel for schedule(static)
        for (int32_t i = 0; i < n; ++i) {
            uint32_t *rowi = M + (int64_t)i * n;
            const uint32_t dik = rowi[k];
            for (int32_t j = 0; j < n; ++j) {
                uint32_t t = oplus(dik, rowk[j]);
                if (t < rowi[j]) rowi[j] = t;
            }
        }
    }
    return 0;
}

/* Dense Dijkstra from one source: dist[v] = SPD(src, v). */
static void dijkstra_one(int32_t n, const uint32_t *A, int32_t src, uint32_t *dist,
                         unsigned char *done)
{
    for (int32_t v = 0; v < n; ++v) { dist[v] = ORACLE_INF; done[v] = 0; }
    dist[src] = 0;
    for (int32_t it = 0; it < n; ++it) {
        int32_t u = -1;
        uint32_t best = ORACLE_INF;
        for (int32_t v = 0; v < n; ++v)
            if (!done[v] && dist[v] < best) { best = dist[v]; u = v; }
        if (u < 0) break;               /* every remaining node is unreachable */
        done[u] = 1;
        const uint32_t *rowu = A + (int64_t)u * n;
        for (int32_t v = 0; v < n; ++v) {
            if (done[v]) continue;
            uint32_t t = oplus(best, rowu[v]);
            if (t < dist[v]) dist[v] = t;
        }
    }
}

/*
 * Rows srcs[0..m-1] of the APSP matrix by Dijkstra: out[r][v] = SPD(srcs[r], v).
 * A is the adjacency (diagonal ignored: a self-loop never shortens a path).
 */
int oracle_dijkstra_rows(int32_t n, const int32_t *A, const int32_t *srcs, int32_t m,
                         int32_t *out, int nthreads)
{
    if (n < 0 || m < 0 || (m > 0 && (!A || !srcs || !out))) return -1;
    for (int32_t r = 0; r < m; ++r)
        if (srcs[r] < 0 || srcs[r] >= n) return -1;
    set_threads(nthreads);
    int bad = 0;
#pragma omp parallel
    {
        unsigned char *done = (unsigned char *)malloc((size_t)(n > 0 ? n : 1));
        if (!done) {
#pragma omp atomic write
            bad = 1;
        }
#pragma omp for schedule(dynamic, 1)
        for (int32_t r = 0; r < m; ++r) {
            if (done)
                dijkstra_one(n, (const uint32_t *)A, srcs[r],
                             (uint32_t *)out + (int64_t)r * n, done);
        }
        free(done);
    }
    return bad ? -1 : 0;
}
