// The no-allocation search, for callers that cannot allocate memory during
// a query (code under HIP graph capture, tight serving loops, harnesses that
// forbid it).
//
// gts_search_noalloc runs the batched form of gts_search with every
// intermediate buffer carved from `scratch`, a file-scope device array of
// kScratchBytes that each GPU the library runs on holds until the process
// ends, and writes the answers into caller-owned device buffers.  The pinned
// host staging it needs is made when the index is built.  The call makes no
// hipMalloc, hipFree, hipHostMalloc or other allocating runtime call.
//
// The array keeps the last call's contents; every buffer a search reads
// before writing (counters, cursors, masks) is cleared by the search itself.
// All calls of a process share the array on a GPU: overlapping calls would
// race, so the calls of this process are serialised by a mutex held until
// the call's answers are complete.
#include <mutex>

#include "gts_internal.h"

namespace {

constexpr size_t kScratchBytes = (size_t)128 << 20;
constexpr int kMaxDevices = 64;

__device__ __align__(256) uint8_t scratch[kScratchBytes];

std::mutex g_mu;                      // one no-allocation call at a time in this process
void *g_scratch[kMaxDevices] = {};    // device address of `scratch` on each device (host stand-in unusable)

// The device address of `scratch` on the current device, looked up once per
// device (each device holds its own copy at its own address).  Caller holds g_mu.
uint8_t *scratch_on_device()
{
    int dev = 0;
    GTS_HIP(hipGetDevice(&dev));
    GTS_CHECK(dev >= 0 && dev < kMaxDevices, GTS_ENOTSUP, "device ordinal beyond the no-allocation table");
    if (!g_scratch[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || p == nullptr)
            gts::fail(GTS_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch[dev] = p;
    }
    return static_cast<uint8_t *>(g_scratch[dev]);
}

}  // namespace

extern "C" gts_status gts_search_noalloc(gts_index *idx, const gts_objects *Q, const float *radius, const int32_t *k,
                                         const gts_query_opts *opts, int64_t *out_offsets, int64_t *out_ids,
                                         void *out_dist, int64_t out_capacity, int64_t *out_total)
{
    return gts::run_guarded([&] {
        GTS_CHECK(idx != nullptr, GTS_EINVAL, "null index");
        GTS_CHECK(Q != nullptr, GTS_EINVAL, "null queries");
        std::lock_guard<std::mutex> lk(g_mu);
        gts::Arena arena;
        arena.base = scratch_on_device();
        arena.size = kScratchBytes;
        gts::QueryCtx *cx = &idx->ctx_na;
        // every buffer is carved afresh; the views are dropped again on exit
        struct Views {
            gts::QueryCtx *c;
            ~Views()
            {
                for (gts::DevBuf &w : c->ws) w.release();
                c->arena = nullptr;
            }
        } views{cx};
        for (gts::DevBuf &w : cx->ws) w.release();
        cx->arena = &arena;
        gts::NoAllocOut na{out_offsets, out_ids, out_dist, out_capacity, out_total};
        gts_result res;
        gts::search(idx, cx, Q, radius, k, opts, &res, &na);
    });
}
