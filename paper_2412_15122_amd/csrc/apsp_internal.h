// Internal declarations shared by the library's translation units.
//
// Storage (all slot-indexed, row-major, leading dimension ld = P, where P is
// the capacity rounded up to a multiple of 128):
//   D   distance matrix            D[i][j] = SPD(i, j)
//   A   adjacency                  A[i][j] = d(i, j); A[s][s] = 0 for a live
//                                  slot s, APSP_INF for a dead or unused one
//   AT  transpose of A (directed graphs only), so in-edges are a row
//   light in-edge index: for each slot y up to 64 entries (x, w) of in-edges
//   x -> y sorted by ascending w, a count, and a bound beta[y] such that
//   every in-edge of y that is not listed weighs at least beta[y].
// Dead and unused slots hold APSP_INF in their whole row and column of D and
// A, including the diagonal, which makes them inert in every kernel.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/apsp.h"

namespace apsp {

constexpr uint32_t INF = 1u << 30;
constexpr int TILE = 128;        // Floyd-Warshall block / matrix padding
constexpr int NIN_L = 64;        // light in-edge index entries per node
constexpr int FUSED_GRID = 512;  // resident work-groups of the mask+recompute kernel
constexpr int FUSED_THREADS = 1024;  // threads of a heavy-row work-group
constexpr int RECOMPUTE_STATS = 6;   // rows, flagged, full scans, sweeps, changed, rows changed
constexpr int ROW_CAP = 32;      // flagged columns listed per row (more: a "heavy" row)
constexpr int RECOMPUTE_BLOCKS = 2048;  // work-groups of the per-row recompute (4 waves each)

enum EdgeMode : int32_t { EDGE_NOOP = 0, EDGE_DECREASE = 1, EDGE_INCREASE = 2 };
enum FusedMode : int32_t { FUSED_REMOVE = 0, FUSED_INCREASE = 1 };
enum ErrBits : int32_t { ERR_VALUE = 1 };

// Device control block: per-update decisions and statistics.
struct Ctl {
    int32_t edge_mode;
    int32_t w_old;
    int32_t duv;
    int32_t err;          // sticky error bits
    unsigned long long flagged;
    int32_t rows;
    int32_t full_scans;
    int32_t sweeps;
    int32_t rows_relaxed;
    int32_t scope_r;
    int32_t scope_c;
    int32_t rows_changed; // rows with a flagged pair whose distance changed
    int32_t short_count;  // index lists queued for a rebuild
    int32_t heavy_count;  // rows deferred to the heavy-row pass
    int32_t pad[1];
    unsigned long long changed;  // flagged pairs whose distance changed
};

// Device view of one graph, passed to kernels by value.
struct DevGraph {
    int32_t *D;
    int32_t *A;
    int32_t *AT;          // nullptr for undirected graphs
    int2 *nin;            // [P][NIN_L] (x, w)
    int32_t *nin_cnt;     // [P]
    int32_t *nin_beta;    // [P]
    int32_t *id_of_slot;  // [P], -1 for dead
    Ctl *ctl;
    int64_t ld;
    int32_t P;
    int32_t n_slots;      // slots [0, n_slots) may be live
    int32_t undirected;
    int32_t lim;          // usable index entries (1..NIN_L)
};

// Row y of the in-edge matrix: Min[y][x] = A[x][y].
__host__ __device__ inline const int32_t *in_matrix(const DevGraph &g) {
    return g.undirected ? g.A : g.AT;
}

// ---- launchers (defined next to their kernels) -----------------------------

void launch_fill(int32_t *p, int64_t count, int32_t v, hipStream_t s);
void launch_load_adj(const DevGraph &g, const int32_t *adj, int64_t adj_ld, int32_t n, hipStream_t s);
void launch_transpose(const int32_t *src, int32_t *dst, int64_t ld, int32_t n, hipStream_t s);
void launch_copy_square(int32_t *dst, const int32_t *src, int64_t ld, int32_t n, hipStream_t s);
void launch_iota(int32_t *p, int32_t n, hipStream_t s);

// Floyd-Warshall over slots [0, n): three launches per 128-wide round.
struct Prof;
// Returns the name of a kernel whose launch failed, or nullptr.
const char *launch_fw(const DevGraph &g, int32_t n, hipStream_t s, Prof *prof);

// Light in-edge index.
void launch_nin_build(const DevGraph &g, int32_t first, int32_t count, int32_t only_short, hipStream_t s);
// The end of an edge update, one launch: a tight increase's recompute
// statistics summed (partials of `blocks` work-groups), then the lists of y0
// and y1 (y1 < 0: y0 only) rebuilt if they have shrunk.
void launch_edge_finish(const DevGraph &g, int32_t y0, int32_t y1, const int32_t *partials, int32_t blocks,
                        hipStream_t s);
void launch_select_vec(const int32_t *vals, int32_t n, int32_t exclude, int2 *list, int32_t *cnt,
                       int32_t *beta, hipStream_t s);
// Rebuild the lists queued by a removal (those that fell below NIN_L/2 while
// unlisted in-edges exist).
void launch_nin_rebuild_queue(const DevGraph &g, const int32_t *queue, hipStream_t s);

// Add node.  The scatter also zeroes the per-update counters.
void launch_scatter_weights(const DevGraph &g, const int32_t *w_out, const int32_t *w_in,
                            const int32_t *slot_of_rank, int32_t n_live, int32_t *wo, int32_t *wi,
                            hipStream_t s);
void launch_add_out(const DevGraph &g, const int2 *plist, const int32_t *pcnt, const int32_t *pbeta,
                    const int32_t *wo, int32_t *out, hipStream_t s);
void launch_add_in(const DevGraph &g, int32_t p, const int32_t *wi, int32_t *in, hipStream_t s);
void launch_add_relax(const DevGraph &g, const int32_t *in, const int32_t *out, hipStream_t s);
// Row and column p placed, p registered, p's out-edges entered in the lists.
void launch_add_finish(const DevGraph &g, int32_t p, int32_t new_id, int32_t rank, int32_t *slot_of_rank,
                       const int32_t *in, const int32_t *out, const int32_t *wo, const int32_t *wi, hipStream_t s);

// Remove node / edge increase: mask + exact recompute of the masked pairs.
// Row marks of the mask detection: one byte per group of 8 rows and chunk
// of 256 columns, bit r set when row 8 g + r has a flag in that chunk.
__host__ __device__ inline int32_t mark_pitch(int64_t P) { return (int32_t)((P + 255) / 256); }

struct FusedArgs {
    int32_t mode;         // FusedMode
    int32_t k;            // removed slot (FUSED_REMOVE)
    int32_t w_old;        // FUSED_INCREASE: read from ctl on the device
    const int32_t *col1;  // per-row vectors (see kernel)
    const int32_t *col2;
    const int32_t *row1;
    const int32_t *row2;
    int32_t *scratch;     // FUSED_GRID * 2 * P ints
    int32_t *heavy_rows;  // [P] rows deferred to the heavy-row pass
    int32_t *heavy_epoch; // [P] heavy_epoch[i] == epoch marks row i heavy
    uint32_t *flag_bits;  // [P][P/32] flag bitmap; zero outside a pending mask (its readers clear it)
    uint32_t *row_bits;   // [P/32] rows holding a flag (batched launches); zero between updates
    uint8_t *marks;       // [P/8][mark_pitch(P)] per (8-row group, 256-column chunk): rows with a flag there
    int32_t mark_pitch;
    int32_t *partials;    // [RECOMPUTE_BLOCKS][RECOMPUTE_STATS] per-work-group statistics of the recompute
    int32_t epoch;        // distinct for every mask pass
};
// Removal: counters zeroed, colk[i] = D[i][k], rowk[j] = D[k][j].
void launch_remove_begin(const DevGraph &g, int32_t k, int32_t *colk, int32_t *rowk, hipStream_t s);
// Mask + recompute in two steps: detection, then the recompute -- or, with
// reset_only, just the clearing of the flag words when cold Floyd-Warshall
// replaces the recompute.  launch_mask_recompute returns the number of
// work-groups whose statistics (Phi, |F|, ...) the update's next kernel sums
// into the control block (launch_remove_finish / launch_edge_finish), negated
// when the heavy-row pass did not run (its partials are then not summed).
void launch_mask_detect(const DevGraph &g, const FusedArgs &fa, hipStream_t s);
int32_t launch_mask_recompute(const DevGraph &g, const FusedArgs &fa, int32_t reset_only, hipStream_t s);
void launch_count_flag_rows(const DevGraph &g, const FusedArgs &fa, hipStream_t s);  // Phi -> ctl->rows
// After a removal's recompute: tombstone of slot k, k purged from the light
// lists (short ones queued), rank table shifted (rank_src -> rank_dst).
void launch_remove_finish(const DevGraph &g, int32_t k, int32_t *queue, const int32_t *rank_src, int32_t *rank_dst,
                          int32_t r, int32_t n_live, const int32_t *partials, int32_t blocks, hipStream_t s);

// Edge update.
// The edge decision and the gathers of columns / rows u and v of D.
void launch_edge_begin(const DevGraph &g, int32_t su, int32_t sv, int32_t w, int32_t *colu, int32_t *colv,
                       int32_t *rowu, int32_t *rowv, hipStream_t s);
// The decrease's relaxation or the tight increase's mask, chosen on the
// device (fa: the increase's mask arguments; its vectors serve both).
void launch_edge_sweep(const DevGraph &g, const FusedArgs &fa, int32_t w, hipStream_t s);

// Query / read-out.
void launch_query(const DevGraph &g, int32_t si, int32_t sj, int32_t *out, int32_t *scratch, hipStream_t s);
// Nodes on some / on every shortest si -> sj path.  rank: the n_live live
// slots in ascending-id order; out: 4 + 2 n_live ints; scratch: 4 P ints;
// bfs: 2 P ints for each of 256 work-groups.
void launch_query_nodes(const DevGraph &g, int32_t si, int32_t sj, const int32_t *rank, int32_t n_live,
                        int32_t *out, int32_t *scratch, int32_t *bfs, hipStream_t s);
void launch_gather_compact(const int32_t *src, int64_t ld, int32_t *dst, int64_t dst_ld,
                           const int32_t *slot_of_rank, int32_t n, hipStream_t s);
void launch_edge_scope(const DevGraph &g, int32_t su, int32_t sv, hipStream_t s);

size_t fused_lds_bytes(int32_t P);
size_t nin_build_lds_bytes(int32_t P);
hipError_t configure_kernels();  // raise dynamic-LDS limits once per process

// Kernel ids for per-kernel timing (apsp_profile).
enum KernelId : int32_t {
    KID_FW_PIVOT = 0, KID_FW_PANEL, KID_FW_TILE, KID_NIN_BUILD, KID_NIN_UPDATE,
    KID_ADD_OUT, KID_ADD_IN, KID_ADD_RELAX, KID_ADD_PLACE, KID_GATHER, KID_FUSED,
    KID_TOMBSTONE, KID_EDGE_BEGIN, KID_EDGE_SWEEP, KID_QUERY, KID_MISC, KID_MASK, KID_COUNT
};

// Event-based timing hooks (implemented in the host API unit).
struct Prof {
    void begin(int32_t kid);
    void end();
    bool on = false;
    void *impl = nullptr;
};

}  // namespace apsp
