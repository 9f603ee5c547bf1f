// The batched kernels for minimax (bottleneck) paths: the same source
// compiled with the (min, max) semiring, in namespace apsp::mm.
#define APSP_SEMIRING_MINIMAX 1
#include "batch.hip"
