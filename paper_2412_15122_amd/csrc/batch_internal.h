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
    int32_t item_begin, item_end;
    int32_t index;      // position in the caller's graphs array
    int32_t pad;
};

struct BatchHeader {
    int32_t num_graphs;
    int32_t counter;     // next position of `order` to take; cleared before each launch
    long long *times;    // [2 * caller's graph count]: wall clock at start / end of each graph
    int32_t pad[60];
};

constexpr int BATCH_THREADS = 256;
constexpr int BATCH_MAX_CAPACITY = APSP_BATCH_MAX_CAPACITY;  // keeps the select stage in LDS

size_t batch_lds_bytes(int32_t P_max);
hipError_t configure_batch();  // raise the dynamic-LDS limit once per process
// Persistent launch of `grid` work-groups over the graphs listed in `order`.
hipError_t launch_batch(BatchHeader *hdr, const BatchGraph *graphs, const int32_t *order, const BatchItem *items,
                        int32_t P_max, int32_t grid, int32_t variant, hipStream_t s);

}  // namespace apsp
