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
constexpr int RECOMPUTE_BLOCKS = 2048;  // work-groups of the per-row recompute
constexpr int RECOMPUTE_WAVES = 4;      // wavefronts per recompute work-group, one row each at a time

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
    int32_t widest;       // widest-path graph: weights stored as WIDEST_TOP - capacity (see widest_xf)
};

// Widest (maximum-capacity) paths run as minimax paths over transformed
// weights: a capacity c in [0, WIDEST_TOP] is stored as WIDEST_TOP - c, so
// the largest over paths of the smallest capacity is WIDEST_TOP minus the
// least over paths of the largest stored weight.  INF (no edge / no path)
// maps to itself; the map is its own inverse on [0, WIDEST_TOP].
constexpr uint32_t WIDEST_TOP = INF - 1;
__host__ __device__ inline int32_t widest_xf(int32_t v) {
    return (uint32_t)v <= WIDEST_TOP ? (int32_t)(WIDEST_TOP - (uint32_t)v) : v;
}

// Row y of the in-edge matrix: Min[y][x] = A[x][y].
__host__ __device__ inline const int32_t *in_matrix(const DevGraph &g) {
    return g.undirected ? g.A : g.AT;
}

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
struct Prof;

// ---- semirings -------------------------------------------------------------
// The kernel sources (fw.hip, update.hip, query.hip and device_common.h) are
// compiled twice: as they are, for shortest paths -- the (min, +) semiring,
// a (+) b = a + b -- in namespace apsp, and with APSP_SEMIRING_MINIMAX defined, for
// minimax (bottleneck) paths -- the (min, max) semiring, a (+) b = max(a, b)
// -- in namespace apsp::mm.  Every distance concatenation in them goes
// through cat(); everything else is shared.
#ifdef APSP_SEMIRING_MINIMAX
#define APSP_SR_BEGIN namespace mm {
#define APSP_SR_END }
#else
#define APSP_SR_BEGIN
#define APSP_SR_END
#endif

APSP_SR_BEGIN
// Path concatenation a (+) b of this unit's semiring.  Entries are at most
// INF: a sum stays below 2^31 (no wrap), and a (+) b >= INF whenever either
// side is INF.
#ifdef APSP_SEMIRING_MINIMAX
__device__ __forceinline__ uint32_t cat(uint32_t a, uint32_t b) { return max(a, b); }
#else
__device__ __forceinline__ uint32_t cat(uint32_t a, uint32_t b) { return a + b; }
#endif
APSP_SR_END

#include "launchers.inc"
namespace mm {
#include "launchers.inc"
// Minimax path query: breadth-first search from si over edges of weight
// <= D[si][sj], one launch per level, a host sync every few levels through
// probe_host (pinned, >= 8 ints).  out as for launch_query.  Returns the
// name of a failed step, or nullptr.
const char *launch_query_bottleneck(const DevGraph &g, int32_t si, int32_t sj, int32_t *out, int32_t *scratch,
                                    int32_t *probe_host, hipStream_t s);
// Minimax pair node sets (output as launch_query_nodes, plus n_slots marks
// after it: 4 + 2 n_live + n_slots ints); scratch: 4 P ints for the search;
// work: 5 P + 1 ints.  Synchronous.
const char *launch_query_nodes_bottleneck(const DevGraph &g, int32_t si, int32_t sj, const int32_t *rank,
                                          int32_t n_live, int32_t *out, int32_t *scratch, int32_t *work,
                                          int32_t *probe_host, hipStream_t s);
}

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
