// Device-side records of a batched launch: one BatchGraph per graph, the
// graph's updates as a contiguous run of BatchItems (applied in order), and a
// header holding the graph count and the work counter the persistent
// work-groups pop from.
#pragma once
#include "apsp_internal.h"

namespace apsp {

enum BatchOp : int32_t { BOP_NONE = 0, BOP_ADD = 1, BOP_REMOVE = 2, BOP_EDGE = 3, BOP_QUERY = 4 };

// Slots, ranks and new ids are resolved on the host before the launch.
//   add     a = new slot p, b = new id, c = live count before the add
//   remove  a = slot k, b = rank of k, c = live count before the removal
//   edge    a = slot u, b = slot v, c = new weight
//   query   a = slot i, b = slot j; out receives 3 + path ints
struct BatchItem {
    int32_t op;
    int32_t n_slots;  // slots that may be live while this update runs
    int32_t a, b, c;
    int32_t pad;
    int32_t *rank_src;    // slot of each rank before the update
    int32_t *rank_dst;    // remove: slot of each rank after it
    const int32_t *w_out; // add: out-edge weights by rank
    const int32_t *w_in;  // add (directed): in-edge weights by rank
    int32_t *out;         // query result
};

struct BatchGraph {
    DevGraph g;
    int32_t *wo, *wi, *vout, *vin, *colu, *colv, *rowu, *rowv;
    int2 *plist;
    int32_t *plist_cnt, *plist_beta;
    int32_t *scratch;   // 4 waves x 2 P: lists of rows with many flags
    int32_t *qscratch;  // 4 P: query candidates
    int32_t *queue;     // P: index lists to rebuild
    uint32_t *flag_bits, *row_bits;
    int32_t *heavy_rows;  // P: lockstep rows deferred to the one-work-group-per-row pass
    int32_t item_begin, item_end;
    int32_t index;      // position in the caller's graphs array
    int32_t pad;
};

struct BatchHeader {
    int32_t num_graphs;
    int32_t counter;     // work queue: next position of `order` to take; cleared before each launch
    long long *times;    // [2 * caller's graph count]: wall clock at start / end of each graph
    int32_t steps;       // lockstep: items per graph at most
    int32_t p_max;       // lockstep: largest pitch of the batch
    int32_t err;         // lockstep: set when a grid barrier wait timed out
    int32_t heavy_claim; // lockstep: next deferred heavy row to take (zero between steps)
    int32_t sweep_claim; // lockstep: next chunk of the row sweeps to take (zero between steps)
    int32_t pad0[23];
    unsigned bar_count;  // lockstep grid barrier (each counter on its own 128-byte line)
    unsigned pad1[31];
    unsigned bar_gen;
    unsigned pad2[31];
    unsigned bar_group[8 * 32];
    long long phase_ts[96];  // lockstep: wall clock after the barriers of the first 32 steps (diagnostics)
    long long work_ts[96];   // lockstep: latest end of a work-group's recompute work, per step (diagnostics)
};

constexpr int BATCH_PHASE_STAMPS = 96;
constexpr int BATCH_RECOMPUTE_ROWS = 16;  // rows per chunk of the lockstep recompute phase
// lockstep tables per step, G + 1 words each: chunk prefixes of the add
// vectors, the sweeps and the recompute, then the graph order of the sweep
// and recompute prefixes (their position k -> graph index)
constexpr int BATCH_TABLES = 4;

// Work-group chunks of an add's vector phase: 256 columns of the new row,
// then (directed) ADD_IN_ROWS rows of the new column.
constexpr int32_t ADD_IN_ROWS = 64;
__host__ __device__ inline int32_t add_out_chunks(int32_t n) { return (n + 255) / 256; }
__host__ __device__ inline int32_t add_vec_chunks(int32_t n, bool undirected) {
    return add_out_chunks(n) + (undirected ? 0 : (n + ADD_IN_ROWS - 1) / ADD_IN_ROWS);
}

constexpr int BATCH_THREADS = 256;
constexpr int BATCH_MAX_CAPACITY = APSP_BATCH_MAX_CAPACITY;  // keeps the select stage in LDS

// Rows per chunk of a lockstep row sweep: about 64K entries (rows of n).
__host__ __device__ inline int32_t batch_rows_per_chunk(int32_t n) {
    const int32_t r = n > 0 ? ((1 << 16) / n) & ~15 : 16;
    return r < 16 ? 16 : r;  // a multiple of 16: a wavefront's rows share a word of row marks
}

// Lockstep row sweeps copy a chunk's row vectors (2 x P_max words) and its
// rows' test values (2 x LOCKSTEP_STAGE_ROWS words) to LDS when the batch's
// largest pitch keeps that small; a chunk holds at most min(rows per chunk,
// n) <= 256 rows (rows per chunk <= 65536 / n).
constexpr int32_t LOCKSTEP_STAGE_ROWS = 256;
constexpr int32_t LOCKSTEP_STAGE_MAX_PITCH = 4608;
__host__ __device__ inline bool lockstep_stages_sweeps(int32_t P_max) { return P_max <= LOCKSTEP_STAGE_MAX_PITCH; }
constexpr int LOCKSTEP_LIGHT_WORDS = ROW_CAP * ROW_CAP + 2 * 64 + 3 * ROW_CAP;  // light_row's per-wave LDS
// The recompute phase's light rows keep their values in LDS (light_row)
// when the launch can hold each wavefront's LIGHT_ROW_WORDS past the
// staging area and still fit three work-groups in a CU's 160 KiB.
__host__ __device__ inline int32_t lockstep_light_offset(int32_t P_max) {
    return 2 * P_max + 2 * LOCKSTEP_STAGE_ROWS;
}
__host__ __device__ inline bool lockstep_light_rows(int32_t P_max) {
    return lockstep_stages_sweeps(P_max) &&
           ((size_t)lockstep_light_offset(P_max) + 4 * (size_t)LOCKSTEP_LIGHT_WORDS) * 4 <= 163840 / 3;
}

#include "batch_launchers.inc"
namespace mm {
#include "batch_launchers.inc"
}

}  // namespace apsp
