// The edge update for callers that cannot allocate (apsp_update_edge_noalloc):
// the same kernels as apsp_update_edge, with the update's working memory --
// gathered vectors, heavy-row scratch, flag bitmap, row bits and marks,
// recompute partials -- in one file-scope device array instead of the
// graph's buffer.  Nothing here allocates: the array is part of the loaded
// code object (one copy per device, held until the process ends), and its
// device address is looked up once per device.
#include <atomic>
#include <mutex>
#include <string>

#include "apsp_internal.h"
#include "host_graph.h"

using namespace apsp;
using namespace apsp_host;

namespace {

// Byte layout of the working memory of an edge update on a graph of pitch P
// (every region 256-byte aligned), in the order EdgeScratch lists it.  The
// array holds the layout of the largest pitch; smaller graphs use the start
// of each region.
struct NoallocLayout {
    size_t colu, colv, rowu, rowv, fscratch, heavy_rows, heavy_epoch, flag_bits, row_bits, marks, partials, total;
};

constexpr size_t al(size_t x) { return (x + 255) & ~(size_t)255; }

constexpr NoallocLayout noalloc_layout(size_t P) {
    NoallocLayout L{};
    size_t off = 0;
    L.colu = off, off = al(off + P * 4);
    L.colv = off, off = al(off + P * 4);
    L.rowu = off, off = al(off + P * 4);
    L.rowv = off, off = al(off + P * 4);
    L.fscratch = off, off = al(off + (size_t)FUSED_GRID * 2 * P * 4);
    L.heavy_rows = off, off = al(off + P * 4);
    L.heavy_epoch = off, off = al(off + P * 4);
    L.flag_bits = off, off = al(off + P * ((P + 31) / 32) * 4);
    L.row_bits = off, off = al(off + ((P + 31) / 32) * 4);
    L.marks = off, off = al(off + (P / 8) * ((P + 255) / 256));
    L.partials = off, off = al(off + ((size_t)RECOMPUTE_BLOCKS * RECOMPUTE_STATS + 2 * (size_t)FUSED_GRID) * 4);
    L.total = off;
    return L;
}

static_assert(APSP_NOALLOC_MAX_CAPACITY % TILE == 0, "the no-allocation limit must be a tile multiple");
constexpr size_t SCRATCH_BYTES = noalloc_layout(APSP_NOALLOC_MAX_CAPACITY).total;

constexpr int MAX_DEVICES = 64;

}  // namespace

// The working memory itself.  In host code `scratch` names a host-side
// stand-in, not the device array: only the address from hipGetSymbolAddress
// (scratch_on) is passed to kernels or fills.
static __device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];

namespace {

struct DeviceScratch {
    std::once_flag once;
    hipError_t status = hipErrorNotInitialized;
    unsigned char *ptr = nullptr;
    // epochs of the heavy-row marks in this device's array: they must not
    // repeat while stale marks hold an earlier value
    std::atomic<int32_t> epoch{0};
};

DeviceScratch g_dev[MAX_DEVICES];

// The device address of `scratch` on `dev`, looked up once per device with
// that device current (the caller's current device is restored).
apsp_status scratch_on(int dev, unsigned char **out) {
    if (dev < 0 || dev >= MAX_DEVICES) return fail(APSP_E_DEVICE, "apsp_update_edge_noalloc: device index out of range");
    DeviceScratch &d = g_dev[dev];
    std::call_once(d.once, [&] {
        int cur = -1;
        hipError_t e = hipGetDevice(&cur);
        if (e == hipSuccess && cur != dev) e = hipSetDevice(dev);
        void *p = nullptr;
        if (e == hipSuccess) e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur >= 0 && cur != dev) (void)hipSetDevice(cur);
        d.status = e;
        d.ptr = e == hipSuccess ? static_cast<unsigned char *>(p) : nullptr;
    });
    if (d.status != hipSuccess || !d.ptr)
        return fail(APSP_E_DEVICE, std::string("apsp_update_edge_noalloc: address of the static scratch array: ") +
                                       hipGetErrorString(d.status));
    *out = d.ptr;
    return APSP_OK;
}

}  // namespace

extern "C" size_t apsp_noalloc_scratch_bytes(void) { return SCRATCH_BYTES; }

extern "C" apsp_status apsp_update_edge_noalloc(apsp_graph *g, int32_t u, int32_t v, int32_t w) {
    int32_t su, sv;
    if (apsp_status bad = check_edge_args(g, "apsp_update_edge_noalloc", u, v, w, &su, &sv)) return bad;
    if (g->cap > APSP_NOALLOC_MAX_CAPACITY)
        return fail(APSP_E_CAPACITY, "apsp_update_edge_noalloc: graph capacity " + std::to_string(g->cap) +
                                         " above the static scratch limit APSP_NOALLOC_MAX_CAPACITY (" +
                                         std::to_string(APSP_NOALLOC_MAX_CAPACITY) + "); use apsp_update_edge");
    hipPointerAttribute_t attr{};
    if (!hip_ok(hipPointerGetAttributes(&attr, g->base), "apsp_update_edge_noalloc: device of the graph buffer"))
        return APSP_E_DEVICE;
    unsigned char *base = nullptr;
    if (apsp_status st = scratch_on(attr.device, &base)) return st;
    DeviceScratch &d = g_dev[attr.device];

    // every region at its place for the largest pitch, whatever this graph's
    // pitch: a region only ever holds its own kind of data across calls
    const size_t P = (size_t)g->P;
    constexpr NoallocLayout L = noalloc_layout(APSP_NOALLOC_MAX_CAPACITY);
    EdgeScratch sc{};
    sc.colu = reinterpret_cast<int32_t *>(base + L.colu);
    sc.colv = reinterpret_cast<int32_t *>(base + L.colv);
    sc.rowu = reinterpret_cast<int32_t *>(base + L.rowu);
    sc.rowv = reinterpret_cast<int32_t *>(base + L.rowv);
    sc.fscratch = reinterpret_cast<int32_t *>(base + L.fscratch);
    sc.heavy_rows = reinterpret_cast<int32_t *>(base + L.heavy_rows);
    sc.heavy_epoch = reinterpret_cast<int32_t *>(base + L.heavy_epoch);
    sc.flag_bits = reinterpret_cast<uint32_t *>(base + L.flag_bits);
    sc.row_bits = reinterpret_cast<uint32_t *>(base + L.row_bits);
    sc.marks = base + L.marks;
    sc.partials = reinterpret_cast<int32_t *>(base + L.partials);

    // The array keeps what the last call on this device left.  The update
    // needs a clear flag bitmap and clear row bits (its mask stores only
    // nonzero words); they are cleared here by fill kernels (no memset
    // nodes, so the call can be captured).  Heavy-row marks need epochs
    // that never repeat: on wrap-around the marks are cleared and the epochs
    // start again.
    const size_t words = P * ((P + 31) / 32);
    launch_fill(reinterpret_cast<int32_t *>(sc.flag_bits), (int64_t)words, 0, g->stream);
    launch_fill(reinterpret_cast<int32_t *>(sc.row_bits), (int64_t)((P + 31) / 32), 0, g->stream);
    int32_t ep = d.epoch.fetch_add(1) + 1;
    if (ep <= 0 || ep == INT32_MAX) {
        launch_fill(sc.heavy_epoch, (int64_t)APSP_NOALLOC_MAX_CAPACITY, 0, g->stream);
        d.epoch.store(1);
        ep = 1;
    }
    sc.epoch = ep;
    if (apsp_status st = check_launch("apsp_update_edge_noalloc: scratch clear")) return st;

    // profiling events are created on demand: off for this call
    const bool prof_on = g->prof.on;
    g->prof.on = false;
    apsp_status st = update_edge_with(g, "apsp_update_edge_noalloc", u, v, w, sc);
    g->prof.on = prof_on;
    return st;
}
