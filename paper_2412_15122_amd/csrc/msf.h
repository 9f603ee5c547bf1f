// The spanning-forest route of a node removal or a tight edge increase on an
// undirected minimax graph (msf.hip): working memory, carved from the
// heavy-row scratch of the graph (idle until the mask route would use it),
// and launchers.
#pragma once
#include "apsp_internal.h"

namespace apsp {

constexpr int32_t MSF_DMAX = 64;            // pieces (k's degree in the forest) handled; more: the mask route
constexpr int32_t MSF_MAX_PITCH = 32768;    // slots fit the 16-bit halves of an edge key and LDS
constexpr int32_t MSF_MAX_HOOK_WALK = 64;   // hooks followed per relabel; deeper: the mask route
constexpr int32_t MSF_INFO = 64;

// info[] words
enum MsfInfo : int32_t {
    MI_TREE = 0,    // forest edges found
    MI_HOOKS = 1,   // hooks in the current round
    MI_ACTIVE = 2,  // rounds still running
    MI_FAIL = 3,    // MSF_FAIL_* bits
    MI_D = 4,       // pieces of T - k (T - e for a raised edge e: 2, or 0 when e is not in T)
    MI_SMALL = 5,   // nodes outside the largest piece
    MI_GIANT = 6,   // index of the largest piece
    MI_COMP = 7,    // nodes of k's component other than k
};
enum MsfFail : int32_t {
    MSF_FAIL_CERT = 1,    // an unlisted edge could be lighter than a forest edge
    MSF_FAIL_SPAN = 2,    // the forest does not span a component of G
    MSF_FAIL_DEEP = 4,    // a hook chain longer than MSF_MAX_HOOK_WALK
    MSF_FAIL_DEGREE = 8,  // more than MSF_DMAX pieces
    MSF_FAIL_STATE = 16,  // an inconsistency (never expected)
};

struct MsfWork {
    int32_t *label, *hook;            // component of each slot; hook of each root
    unsigned long long *best;         // lightest outgoing index edge per root
    int32_t *tree_a, *tree_b, *tree_w;  // forest edges
    int32_t *comp_max, *comp_size;    // heaviest forest edge and size per component
    int32_t *pidx;                    // piece of each node of k's component (-1 elsewhere)
    int32_t *small;                   // nodes outside the largest piece
    uint32_t *rowchg;                 // rows with a changed entry
    int32_t *info;                    // MsfInfo
    int32_t *psize;                   // piece sizes
    unsigned long long *table;        // lightest edge between pieces [MSF_DMAX][MSF_DMAX]
    int32_t *xab, *yab, *wab;         // per piece pair: exit node, entry node, largest weight on the way
    int64_t ints;                     // words used
};

MsfWork msf_work(int32_t *scratch, int32_t P);
hipError_t msf_configure();
// Boruvka rounds over the light index, the certificate, the pieces of T - k;
// with k < 0, of T - (eu, ev) for an edge raised from weight ew (the forest is
// the one of the graph before the change).  eu < 0: no such edge.
void launch_msf_forest(const DevGraph &g, const MsfWork &w, int32_t k, int32_t eu, int32_t ev, int32_t ew,
                       int32_t rounds, hipStream_t s);
// Replacement edges, the pieces' forest, the new entries of the small pieces'
// rows (and their mirrors), Phi'.
void launch_msf_update(const DevGraph &g, const MsfWork &w, int32_t small_count, hipStream_t s);

}  // namespace apsp
