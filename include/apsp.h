/*
 * apsp.h -- C ABI of the warm-start all-pairs shortest-path library (gfx950).
 *
 * The library keeps the APSP matrix of a dense weighted graph resident on
 * one GPU and updates it exactly after a minor change, following the paper
 * "Solving the all pairs shortest path problem after minor update of a
 * large dense graph" (Liu, arXiv 2412.15122):
 *
 *   apsp_cold          cold APSP (Floyd-Warshall; Section 1)
 *   apsp_add_node      G + p   (Theorems 1, 2 and 3 and
 *                               Corollaries 1 and 2; Sec. 3.1)
 *   apsp_remove_node   G - G_k (need_update_list by Theorem 4 /
 *                               Corollary 3, then recompute of the
 *                               listed pairs; Section 3.2, Algorithm 5)
 *   apsp_update_edge   one edge raised or lowered (Section 3.3, Algorithm 6;
 *                               done directly, see each call)
 *   apsp_query         warm single-pair shortest path (Section 4, Alg. 7)
 *   apsp_query_nodes   nodes on some / on every shortest path of a pair
 *                      (Algorithms 8 and 10)
 *
 * Values.  Weights and distances are int32 in [0, APSP_INF]; APSP_INF
 * (2^30) means "no edge" / "unreachable".  Path lengths saturate at
 * APSP_INF.  The diagonal of an adjacency matrix is ignored and taken as 0.
 * Every result is bit-exact: it equals the cold APSP matrix of the updated
 * graph.
 *
 * Ids.  A graph created with n nodes has ids 0..n-1.  apsp_add_node gives
 * the new node id max_id + 1 (the paper appends node N + 1); a removed id is
 * never reused.  Vectors indexed by node and matrices read back are in
 * ascending-id order (the paper's index order).
 *
 * Memory.  The caller owns all device memory: one buffer of
 * apsp_required_bytes(capacity, kind) bytes, 256-byte aligned, passed to
 * apsp_cold and kept alive until apsp_graph_destroy.  The library carves
 * the distance matrix, the adjacency (and its transpose for directed
 * graphs), an index of light in-edges and its workspace out of it; it never
 * allocates or frees device memory itself.  Pointers whose name ends in
 * _dev are device pointers; all others are host pointers.
 *
 * Streams.  Every call enqueues on the graph's HIP stream (given to
 * apsp_cold, changeable with apsp_set_stream) and returns without waiting,
 * except the calls documented as synchronous.
 *
 * Errors.  Calls return an apsp_status; nothing is thrown across the ABI.
 * Arguments are checked before anything is enqueued, so a call that returns
 * an error leaves the graph unchanged.  Values that live in device memory
 * (adjacency entries, weight vectors) are checked on the device: an entry
 * outside [0, APSP_INF] is treated as an absent edge and the graph records
 * a sticky error that apsp_sync returns (once) as APSP_E_VALUE.  APSP_E_DEVICE means a HIP
 * call failed and the device state is undefined; rebuild with apsp_cold.
 * apsp_last_error() gives a message for the last failing call on the
 * calling thread.
 *
 * Threads.  A graph handle must not be used by two threads at once.
 */
#ifndef APSP_H
#define APSP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define APSP_INF 1073741824
#define APSP_ABI_VERSION 1
/* Largest capacity (node slots) of one graph. */
#define APSP_MAX_CAPACITY 38272

typedef enum {
    APSP_OK = 0,
    APSP_E_INVALID = -1,   /* bad argument; nothing enqueued */
    APSP_E_NOT_FOUND = -2, /* id is not live */
    APSP_E_CAPACITY = -3,  /* no free slot, buffer too small, or output too short */
    APSP_E_DEVICE = -5,    /* HIP failure; device state undefined */
    APSP_E_VALUE = -7      /* sticky: a device-resident weight was out of range */
} apsp_status;

/* Graph kind: directed or undirected, optionally OR-ed with APSP_MINIMAX.
 * APSP_MINIMAX selects minimax (bottleneck) paths, the (min, max) semiring:
 * D[i][j] = the least, over walks from i to j, of the largest edge weight on
 * the walk (0 when i == j), the variant the paper's discussion section says
 * its algorithms carry over to.  Every single-graph call then runs the same
 * steps with max in place of + (Theorems 1–3 and Corollary
 * 3 hold with max, which is monotone with 0 as identity on weights
 * >= 0).  A batch (apsp_batch_run) takes graphs of one kind: all minimax
 * (widest graphs included) or none.
 *
 * APSP_WIDEST (instead of APSP_MINIMAX) selects widest paths, the (max, min)
 * semiring the discussion section names beside minimax paths: weights are
 * capacities c in [0, APSP_INF - 1] (APSP_INF: no edge), and
 * W[i][j] = the largest, over walks from i to j, of the smallest capacity
 * on the walk; W[i][i] = APSP_INF - 1, and W[i][j] = APSP_INF when j is
 * unreachable.  The library stores each capacity c as the weight
 * (APSP_INF - 1) - c and runs the minimax kernels: a walk's smallest
 * capacity is APSP_INF - 1 minus its largest stored weight, so
 * W[i][j] = (APSP_INF - 1) - D[i][j] for the minimax matrix D of the stored
 * weights, exactly.  Every value crossing the boundary is converted: the
 * adjacency and add-node capacities on the way in, edge-update capacities,
 * and matrices, adjacency read-outs and query distances (single or batched)
 * on the way out.  Paths and node sets are those of the minimax problem,
 * which are the widest paths. */
typedef enum { APSP_DIRECTED = 0, APSP_UNDIRECTED = 1, APSP_MINIMAX = 2, APSP_WIDEST = 4 } apsp_kind;

/* What apsp_remove_node and an edge increase do after building the mask
 * (Algorithm 5 switches to Floyd-Warshall when Cost exceeds delta). */
typedef enum {
    APSP_FALLBACK_NEVER = 0,  /* always recompute the masked pairs (default) */
    APSP_FALLBACK_COST = 1,   /* Algorithm 5: cold FW on G' when Cost > delta;
                                 the decision reads Phi back (synchronous) */
    APSP_FALLBACK_ALWAYS = 2  /* always cold FW on G' */
} apsp_fallback;

/* How apsp_import checks the matrix it is given. */
typedef enum {
    APSP_IMPORT_TRUSTED = 0,  /* only the O(n^2) checks of a distance matrix */
    APSP_IMPORT_EXACT = 1     /* also a cold recompute, compared entry by entry */
} apsp_import_check;

typedef struct apsp_graph apsp_graph;

/* Per-update statistics of the last update (apsp_last_stats). */
typedef struct {
    int64_t flagged;     /* |F|: pairs in the need_update mask */
    int32_t rows;        /* Phi: rows with at least one flagged pair */
    int32_t n_before;    /* live node count before the update */
    double cost;         /* Definition 1: Phi / (N - 1) */
    int32_t kind;        /* 0 none, 1 add, 2 remove, 3 decrease, 4 increase */
    int32_t noop;        /* 1 when D provably did not change (O(1) path) */
    int32_t fallback;    /* 1 when cold Floyd-Warshall ran instead */
    int32_t full_scans;  /* in-edge scans that went past the light-edge index */
    int32_t sweeps;      /* largest number of relaxation sweeps of one row */
    int32_t rows_relaxed;/* rows touched by an add-node / decrease relaxation */
    int32_t heavy_rows;  /* rows with more than 32 flagged pairs (one work-group each) */
    int32_t rows_changed;/* Phi': rows with at least one changed pair */
    int64_t changed;     /* |F'|: flagged pairs whose distance changed -- the
                          * refined need_update list of Algorithms 11 and 12:
                          * by Theorem 6 (and its converse) exactly
                          * the pairs whose every shortest path uses the
                          * removed node (or the raised edge).  0 after a cold
                          * fallback. */
    double cost_refined; /* Phi' / (N - 1) */
    int32_t route;       /* removals and tight increases: 0 mask + recompute; 1 the
                          * minimum-spanning-forest route of an undirected minimax
                          * graph (only the pairs whose distance changes are
                          * written; see apsp_remove_node, apsp_update_edge) */
    int32_t pad;
} apsp_update_stats;

/* ---- sizing ------------------------------------------------------------ */

/* Bytes of device memory a graph of `capacity` node slots needs.
 * Returns 0 for an invalid capacity or kind.  Host only. */
size_t apsp_required_bytes(int32_t capacity, int32_t kind);

/* ---- construction ------------------------------------------------------ */

/* Cold start: build a graph from the n x n adjacency matrix adj_dev
 * (row-major, leading dimension adj_ld >= n, row i = edges out of node i)
 * and compute its APSP matrix by blocked Floyd-Warshall.
 *   kind       APSP_DIRECTED or APSP_UNDIRECTED (adjacency must be
 *              symmetric; asymmetric pairs take the smaller weight and set
 *              the sticky error), either OR-ed with APSP_MINIMAX for
 *              minimax paths
 *   capacity   node slots, n <= capacity <= APSP_MAX_CAPACITY, >= 1
 *   dev_buf    caller-owned device buffer of dev_buf_bytes >=
 *              apsp_required_bytes(capacity, kind), 256-byte aligned
 *   hip_stream hipStream_t to enqueue on (NULL = default stream)
 *   out        receives the handle (host memory owned by the library)
 * n = 0 gives an empty graph.  adj_dev is only read during the call's
 * kernels; it may be freed after the stream has passed them. */
apsp_status apsp_cold(const int32_t *adj_dev, int32_t n, int64_t adj_ld, int32_t kind,
                      int32_t capacity, void *dev_buf, size_t dev_buf_bytes,
                      void *hip_stream, apsp_graph **out);

/* Warm start from a distance matrix that is already known: the premise of
 * the paper's problem statement (Section 1: the old graph's all-pairs
 * shortest-path matrix is given, and only the update is to be paid for).
 * Builds a graph as apsp_cold does from adj_dev, but takes D from apsp_dev
 * (n x n int32, row-major, leading dimension apsp_ld >= n, row i = distances
 * from node i) instead of running Floyd-Warshall: O(n^2) work.
 *   ids      host array of n strictly ascending ids in [0, INT32_MAX) for
 *            rows 0..n-1 (NULL = 0..n-1); read during the call only.
 *   next_id  the id the next apsp_add_node returns (later ones count up
 *            from it), above every id and below INT32_MAX; -1 = the
 *            largest id + 1.  Lets a
 *            copy keep a graph's id sequence (apsp_next_id) when its largest
 *            ids were removed.
 *   verify   APSP_IMPORT_TRUSTED: the checks below only;
 *            APSP_IMPORT_EXACT: also a cold Floyd-Warshall of the adjacency,
 *            compared with apsp_dev entry by entry (a cold start's cost).
 * The checks, always made: every entry in [0, APSP_INF], a zero diagonal,
 * D[i][j] <= adj[i][j], and symmetry for an undirected graph.  A matrix that
 * passes them but is not the distance matrix of adj (possible only under
 * APSP_IMPORT_TRUSTED) makes every later result undefined.
 * The call waits for hip_stream (it reads the check's count back); adj_dev
 * and apsp_dev may be freed when it returns.
 * Errors: as apsp_cold, and APSP_E_INVALID for a bad verify value, bad ids
 * or next_id, or a matrix that fails a check (no handle is made). */
apsp_status apsp_import(const int32_t *adj_dev, int64_t adj_ld, const int32_t *apsp_dev, int64_t apsp_ld,
                        int32_t n, const int32_t *ids, int32_t next_id, int32_t kind, int32_t capacity,
                        void *dev_buf, size_t dev_buf_bytes, void *hip_stream, int32_t verify, apsp_graph **out);

/* Recompute D from the current adjacency by cold Floyd-Warshall (the
 * fallback of Algorithm 5, and recovery).  Asynchronous. */
apsp_status apsp_recompute_cold(apsp_graph *g);

/* Release the handle.  Does not touch the caller's device buffer.  Waits
 * for the graph's stream. */
apsp_status apsp_graph_destroy(apsp_graph *g);

/* ---- updates (asynchronous) ---------------------------------------------- */

/* Add node p (paper: G + p, Section 3.1).  w_out_dev[t] is the weight of
 * p -> t and w_in_dev[t] the weight of t -> p, for the t-th live node in
 * ascending-id order (length = live count before the call).  For an
 * undirected graph w_in_dev may be NULL (it equals w_out_dev).  New row:
 * SPD(p, r) = min_t d(p,t) + SPD(t,r) (Corollary 1); new column:
 * SPD(r, p) = min_t SPD(r,t) + d(t,p) (Corollary 2); old pairs:
 * min(SPD(i,j), SPD(i,p) + SPD(p,j)) (Theorem 3).  *new_id (host)
 * receives max_id + 1.  Returns APSP_E_CAPACITY when every slot is used, or
 * when max_id + 1 would reach INT32_MAX (ids stay below it). */
apsp_status apsp_add_node(apsp_graph *g, const int32_t *w_out_dev, const int32_t *w_in_dev,
                          int32_t *new_id);

/* Remove node `id` (paper: G - G_k, Section 3.2, Algorithm 5).  Pairs (i,j)
 * with D[i][k] + D[k][j] == D[i][j] form the need_update mask (Corollary
 * 3: all others keep their distance); the masked pairs are
 * recomputed exactly on G - G_k, or cold Floyd-Warshall runs, per the
 * fallback policy.  The id is retired.
 * On an undirected minimax (or widest) graph the call first tries the
 * refined set of Algorithms 11-12 (Theorem 6) directly: a minimum spanning
 * forest of G over the light in-edge index, certified against every
 * unlisted edge; only pairs whose forest path crossed k can change, and
 * their new distances follow from the lightest edges joining the pieces the
 * forest falls into.  This writes only the changed pairs.  When the
 * certificate or a size limit (capacity above 32768, k joining more than
 * 64 pieces) rejects it, the mask route runs; both give the same matrix.
 * The route taken is in apsp_update_stats.route.  This call waits once for
 * the device (the certificate's read-back) on such graphs. */
apsp_status apsp_remove_node(apsp_graph *g, int32_t id);

/* Set the weight of edge u -> v (and v -> u for an undirected graph) to w,
 * 0 <= w <= APSP_INF (APSP_INF deletes the edge).  u != v, both live.
 * The paper (Algorithm 6) removes one endpoint and adds it back; this call
 * gets the same D directly: a decrease below D[u][v] relaxes every pair
 * through the new edge (Theorem 3 with a relay node on the edge), an
 * increase of an edge with D[u][v] == w_old recomputes the pairs whose
 * shortest distance can use it (Corollary 3 applied to that relay
 * node); any other change leaves D as it is.  The choice is made on the
 * device: the call never waits, except on an undirected minimax (or widest)
 * graph, where it reads the device's choice back: a tight increase there
 * first tries the spanning-forest route of apsp_remove_node with the raised
 * edge in place of the removed node (the forest of the graph before the
 * change; if the edge is not in it no distance changes, otherwise only the
 * pairs across the two pieces it separates can, and they take their values
 * from the lightest edge now joining the pieces), and waits once more for
 * its certificate; when the certificate or a size limit rejects it, the
 * mask route runs, with the same matrix.  The route taken is in
 * apsp_update_stats.route. */
apsp_status apsp_update_edge(apsp_graph *g, int32_t u, int32_t v, int32_t w);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * update as apsp_update_edge, with the same kernels and bit for bit the
 * same results (on an undirected minimax graph always by the mask route),
 * but its working memory (the gathered columns and rows, the
 * flag bitmap, row marks, heavy-row scratch and recompute partials, which
 * apsp_update_edge keeps in the graph's buffer) is a static array inside
 * the library, apsp_noalloc_scratch_bytes() bytes on every device the
 * library runs on, held until the process ends.  The call allocates
 * nothing (no hipMalloc, hipHostMalloc or event creation; profiling is off
 * for it) and clears the parts that must start at zero with fill kernels.
 * Every call on one device shares that device's array: calls that overlap
 * on one device (another stream, another thread) race and give undefined
 * results; calls ordered on one stream are safe.  Graphs of capacity above
 * APSP_NOALLOC_MAX_CAPACITY get APSP_E_CAPACITY (nothing enqueued); other
 * errors as apsp_update_edge. */
#define APSP_NOALLOC_MAX_CAPACITY 4224
apsp_status apsp_update_edge_noalloc(apsp_graph *g, int32_t u, int32_t v, int32_t w);
/* Bytes of the static working-memory array of apsp_update_edge_noalloc (per device). */
size_t apsp_noalloc_scratch_bytes(void);

/* ---- queries (synchronous) ------------------------------------------------ */

/* Shortest path from i to j (Algorithm 7, Section 4): *dist = D[i][j]; the
 * path is the lexicographically smallest shortest simple path over ids,
 * found among Algorithm 7's candidates {t : D[i][t] + D[t][j] == D[i][j]}
 * (Theorem 5).  With zero-weight edges any shortest simple path
 * may be returned; on a minimax graph (APSP_MINIMAX) the path is a simple
 * path whose largest edge weight is D[i][j], found over the same candidates
 * with max in place of +.  path_ids (host, path_cap entries) receives the ids from
 * i to j; *path_len its length (1 when i == j, 0 when unreachable, in which
 * case *dist = APSP_INF).  If path_cap < *path_len, returns
 * APSP_E_CAPACITY with *dist and *path_len set.  path_ids may be NULL when
 * path_cap is 0. */
apsp_status apsp_query(apsp_graph *g, int32_t i, int32_t j, int32_t *dist,
                       int32_t *path_ids, int32_t path_cap, int32_t *path_len);

/* The nodes of the shortest paths from i to j (Section 4: Algorithm 7's
 * candidates, Theorem 5; Algorithm 8's paths; Algorithm 10's
 * key_node_list).  *dist = D[i][j].
 *   on_ids  (host, on_cap entries): every live t with
 *           D[i][t] + D[t][j] == D[i][j], i and j included -- the nodes that
 *           lie on some shortest walk from i to j (with positive weights, the
 *           union of the node sets of all shortest paths).
 *   key_ids (host, key_cap entries): the nodes other than i and j that every
 *           shortest walk from i to j visits (the intersection of all
 *           shortest paths, i and j taken out), computed exactly -- not from
 *           a subset of the paths.
 * Both ascending; *on_len / *key_len their lengths.  i == j: on = {i},
 * key = {}; unreachable: both empty and *dist = APSP_INF.  If a buffer is
 * too small, returns APSP_E_CAPACITY with *dist and both lengths set.
 * A buffer may be NULL when its cap is 0.  Work: one pass over row i and
 * column j, then O(K^2) adjacency reads for K candidates (more only for
 * levels joined by zero-weight edges).  Uses the graph's update scratch:
 * ordered on the graph's stream like every call.  On a minimax graph
 * (APSP_MINIMAX) the sets are over optimal walks -- those whose edges all
 * weigh at most D[i][j]: on = {t : max(D[i][t], D[t][j]) == D[i][j]}, key =
 * the nodes on every such walk, found as the interior nodes t of one such
 * path for which a search from i over edges <= D[i][j] that avoids t does
 * not reach j (one search per interior node).  Errors: APSP_E_INVALID for
 * NULL outputs, APSP_E_NOT_FOUND for an id that is not live. */
apsp_status apsp_query_nodes(apsp_graph *g, int32_t i, int32_t j, int32_t *dist,
                             int32_t *on_ids, int32_t on_cap, int32_t *on_len,
                             int32_t *key_ids, int32_t key_cap, int32_t *key_len);

/* Algorithm 8's list of shortest i -> j paths (Section 4): the query's own
 * path (apsp_query), then, for every other node t on some shortest i -> j
 * path (the candidate set of apsp_query_nodes) in ascending id order and not
 * on a path already listed through it, the path i -> t followed by
 * t -> j, each distinct path once.  Every listed path is a shortest simple
 * walk (on minimax / widest graphs: an optimal one); the list need not hold
 * every shortest path.  Output (host memory): path q is
 * ids[offsets[q] .. offsets[q + 1]); *npaths paths, *ids_len ids in all;
 * *dist as apsp_query.  i == j gives [[i]]; an unreachable j gives no path
 * (offsets[0] = 0).  The paths run on the device, one work-group per
 * candidate (chunks of up to 128), then one read-back per chunk;
 * synchronous.  APSP_E_CAPACITY when offsets_cap < *npaths + 1 or
 * ids_cap < *ids_len (both sizes are set, nothing else written);
 * APSP_E_NOT_FOUND for a dead id. */
apsp_status apsp_query_paths(apsp_graph *g, int32_t i, int32_t j, int32_t *dist, int32_t *ids, int64_t ids_cap,
                             int64_t *ids_len, int32_t *offsets, int32_t offsets_cap, int32_t *npaths);

/* Copy the live distance matrix (ascending-id order) into out_dev
 * (n x n, leading dimension out_ld >= n).  Asynchronous. */
apsp_status apsp_read_matrix(apsp_graph *g, int32_t *out_dev, int64_t out_ld);

/* Same for the adjacency matrix (diagonal 0). */
apsp_status apsp_read_adjacency(apsp_graph *g, int32_t *out_dev, int64_t out_ld);

/* The id the next apsp_add_node will return: one above the largest id the
 * graph has ever held (ids of removed nodes are not reused).  Host only. */
apsp_status apsp_next_id(const apsp_graph *g, int32_t *id);

/* Live node count (host bookkeeping; never waits). */
apsp_status apsp_node_count(const apsp_graph *g, int32_t *n);

/* Live ids in ascending order into ids (host, cap entries); *n receives the
 * count.  APSP_E_CAPACITY when cap is too small (with *n set). */
apsp_status apsp_node_ids(const apsp_graph *g, int32_t *ids, int32_t cap, int32_t *n);

/* |R| and |C| of edge u -> v at its current weight w: R = {i : D[i][u] + w
 * == D[i][v] < INF}, C = {j : w + D[v][j] == D[u][j] < INF}.  |R| * |C|
 * bounds how many pairs route through the edge.  Synchronous. */
apsp_status apsp_edge_scope(apsp_graph *g, int32_t u, int32_t v, int32_t *r_count,
                            int32_t *c_count);

/* Statistics of the last update.  Synchronous. */
apsp_status apsp_last_stats(apsp_graph *g, apsp_update_stats *out);

/* ---- control --------------------------------------------------------------- */

/* Wait for the graph's stream; returns the sticky device error if any
 * (and clears it). */
apsp_status apsp_sync(apsp_graph *g);

/* Later calls on g enqueue on hip_stream.  Nothing is enqueued: work
 * already queued on g's previous stream is not ordered before the new
 * stream's by the library (the caller orders them, e.g. with an event). */
apsp_status apsp_set_stream(apsp_graph *g, void *hip_stream);

/* Fallback policy of removals and edge increases; delta is Algorithm 5's
 * threshold on Cost (used by APSP_FALLBACK_COST). */
apsp_status apsp_set_fallback(apsp_graph *g, int32_t policy, double delta);

/* Use only the first `limit` entries (1..64) of each node's light in-edge
 * index; entries beyond it are treated as unindexed.  Results do not
 * change; a small limit exercises the exhaustive-scan path.  Default 64. */
apsp_status apsp_set_index_limit(apsp_graph *g, int32_t limit);

/* Per-kernel timing with HIP events on the graph's stream.  kernel_mask has
 * bit k set for every kernel id k (0..apsp_kernel_count()-1) to time; -1
 * times all, 0 stops.  The call waits for the stream and clears the totals.
 * apsp_profile_read waits for the stream and returns, for kernel `kernel`,
 * the number of timed launches and their summed duration in ms. */
apsp_status apsp_profile(apsp_graph *g, int64_t kernel_mask);
apsp_status apsp_profile_read(apsp_graph *g, int32_t kernel, int64_t *launches, double *total_ms);
/* As apsp_profile, but only launches 0, every, 2 every, ... of each kernel in
 * kernel_mask are timed (each timed launch costs two event records on the
 * stream; sampling keeps that cost out of the launches in between).  every
 * >= 1, else APSP_E_INVALID. */
apsp_status apsp_profile_every(apsp_graph *g, int64_t kernel_mask, int32_t every);
int32_t apsp_kernel_count(void);
const char *apsp_kernel_name(int32_t kernel);

/* ---- copies of a graph ------------------------------------------------- */

/* A second handle with the same state as g (matrices, index, ids), in the
 * caller's buffer dev_buf of apsp_required_bytes(capacity of g, kind of g)
 * bytes, enqueued on hip_stream after waiting for g's stream (g's stream
 * then waits for the copy before g's next call).  The copy is independent
 * of g from then on.  Errors as apsp_cold. */
apsp_status apsp_graph_clone(apsp_graph *g, void *dev_buf, size_t dev_buf_bytes, void *hip_stream,
                             apsp_graph **out);

/* A copy of g with `capacity` node slots (at least the slots g has in use,
 * e.g. to add nodes to a full graph), in the caller's buffer dev_buf of
 * apsp_required_bytes(capacity, kind of g) bytes: every used slot keeps its
 * place, its ids, distances, weights and index list, so the copy behaves as
 * g would with more room (same ids, same next id).  O(n^2) device copies,
 * enqueued on hip_stream after g's stream; g's stream then waits for the
 * copy.  g is unchanged.  Errors: APSP_E_INVALID (NULL arguments, capacity
 * below the slots in use or above APSP_MAX_CAPACITY, a misaligned or
 * overlapping buffer), APSP_E_CAPACITY (buffer too small), APSP_E_DEVICE. */
apsp_status apsp_grow(apsp_graph *g, int32_t capacity, void *dev_buf, size_t dev_buf_bytes, void *hip_stream,
                      apsp_graph **out);

/* The caller has copied g's whole buffer (apsp_required_bytes bytes, e.g.
 * out to host memory and back) into dev_buf; from now on g uses dev_buf and
 * the old buffer may be freed.  Nothing is enqueued: the caller orders the
 * copy before g's next call (e.g. on g's stream).  Lets a server move idle
 * graphs out of HBM and back without a cold start.  A graph detached with
 * apsp_graph_detach (below) is usable again after this call. */
apsp_status apsp_graph_relocate(apsp_graph *g, void *dev_buf, size_t dev_buf_bytes);

/* The caller is about to free or reuse g's device buffer, e.g. after copying
 * it to host memory: waits for g's stream, then every call that would touch
 * device memory through g (updates, queries, read-outs, statistics, sync,
 * clone, grow, batches) returns APSP_E_INVALID and enqueues nothing, until
 * apsp_graph_relocate gives g a buffer again.  Host-only calls (ids, counts,
 * apsp_next_id, settings, apsp_graph_destroy) keep working.  Errors:
 * APSP_E_INVALID (NULL), APSP_E_DEVICE (the stream wait failed; g stays
 * attached). */
apsp_status apsp_graph_detach(apsp_graph *g);

/* ---- batched updates --------------------------------------------------- */

/* Many graphs and their queued updates run in one persistent launch: every
 * work-group takes one graph at a time (by default the graph with the most
 * work first) and applies that graph's items in the order they appear in
 * the item array, with the same semantics, and bit for bit the same
 * matrices, as the single calls above (apsp_add_node, apsp_remove_node,
 * apsp_update_edge, apsp_query).  Graphs of a batch need capacity <=
 * APSP_BATCH_MAX_CAPACITY.  The fallback policy is not applied inside a
 * batch: removals and increases always take the masked recompute. */
#define APSP_BATCH_MAX_CAPACITY 16384

typedef enum {
    APSP_OP_ADD_NODE = 1,    /* w_out_dev, w_in_dev as apsp_add_node */
    APSP_OP_REMOVE_NODE = 2, /* u = id */
    APSP_OP_UPDATE_EDGE = 3, /* u -> v gets weight w */
    APSP_OP_QUERY = 4        /* u -> v; the result goes to out_dev */
} apsp_batch_op;

typedef struct {
    int32_t graph;            /* index into the graphs array of apsp_batch_run */
    int32_t op;               /* apsp_batch_op */
    int32_t u, v, w;
    int32_t out_cap;          /* query: int32 slots at out_dev, >= 3 + live nodes */
    const int32_t *w_out_dev; /* add: out-edge weights, one per live node, ascending ids */
    const int32_t *w_in_dev;  /* add, directed graphs: in-edge weights */
    int32_t *out_dev;         /* query: [distance, path length, status (0 ok), path ids...] */
} apsp_batch_item;

typedef struct apsp_batch apsp_batch;

/* Device workspace for batches of up to max_graphs graphs and max_items items. */
size_t apsp_batch_workspace_bytes(int32_t max_graphs, int32_t max_items);
/* ws_dev: caller-owned device buffer of apsp_batch_workspace_bytes bytes,
 * 256-byte aligned, alive until apsp_batch_destroy. */
apsp_status apsp_batch_create(void *ws_dev, size_t ws_bytes, int32_t max_graphs, int32_t max_items,
                              apsp_batch **out);
apsp_status apsp_batch_destroy(apsp_batch *b);
/* Two schedules.  Work queue (variants 0, 1): every work-group takes one
 * graph at a time (order: 0 most work first, 1 array order) and runs all of
 * its items alone.  Lockstep (variants 2, 3, 4): step s applies item s of
 * every graph, the row sweeps of all graphs spread over the whole grid
 * between grid barriers (a cooperative launch of the resident grid; the
 * order is irrelevant).  Variants 0 and 2 keep 4, 1 and 3 keep 8, 4 keeps
 * 16 loads in flight per lane in the streaming loops.  grid: work-groups (0: two per compute unit, at most
 * one per graph for the work queue; all resident ones for lockstep; a
 * lockstep grid is capped at the resident count).  use_graph: 1 records the
 * launch once in a HIP graph and replays it. */
apsp_status apsp_batch_set_config(apsp_batch *b, int32_t grid, int32_t order, int32_t variant,
                                  int32_t use_graph);
/* Runs items[0..num_items) on graphs[0..num_graphs) (distinct handles) on
 * hip_stream.  The graphs are all shortest-path graphs or all minimax ones
 * (APSP_MINIMAX; else APSP_E_INVALID): the launch runs the kernels of that
 * semiring.  Work queued earlier for a graph on another stream must have
 * completed.  Every item is checked first; if one is invalid, nothing runs,
 * no graph changes, and the status names the first bad item.  new_ids
 * (host, num_items, may be NULL) receives the id of each added node and -1
 * for other items.  Returns once the launch is enqueued; query results are
 * in out_dev when the stream reaches that point. */
apsp_status apsp_batch_run(apsp_batch *b, apsp_graph *const *graphs, int32_t num_graphs,
                           const apsp_batch_item *items, int32_t num_items, void *hip_stream,
                           int32_t *new_ids);
/* Waits for the last apsp_batch_run and reports APSP_E_DEVICE if a lockstep
 * grid barrier timed out (every wait is bounded, so a launch always ends;
 * the graphs of such a batch are then in an undefined state). */
apsp_status apsp_batch_status(apsp_batch *b);
/* Per-graph timing of the last apsp_batch_run, read from the device wall
 * clock (synchronous: waits for that run's stream).  start_us[i] / end_us[i]
 * are when a work-group took graphs[i] and finished its items, in
 * microseconds from the earliest start; -1 for graphs without items.
 * num_graphs must equal that run's. */
apsp_status apsp_batch_graph_times(apsp_batch *b, double *start_us, double *end_us, int32_t num_graphs);
/* Diagnostics of the last lockstep apsp_batch_run (synchronous): for each of
 * its first 32 steps, the wall clock (microseconds from the start of the
 * first graph) after the grid barriers ending the per-graph phase, the row
 * sweeps and the recompute (0 where a step had no recompute phase); *count
 * receives min(cap, 3 * steps).  Zero entries for the work-queue schedule. */
apsp_status apsp_batch_phase_times(apsp_batch *b, double *us, int32_t cap, int32_t *count);

const char *apsp_last_error(void);
int32_t apsp_abi_version(void);

#ifdef __cplusplus
}
#endif
#endif /* APSP_H */
