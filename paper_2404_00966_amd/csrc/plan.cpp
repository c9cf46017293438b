// Search plans (gts_plan_* in include/gts.h): the batched processing of
// Sec. 5.1 for a query stream of a fixed shape, recorded once into a HIP
// graph and replayed.
//
// Recording runs the batched search in graph mode on the plan's own stream
// under stream capture: the per-query radius and k come from device arrays,
// every intermediate buffer is carved from the plan's fixed space in the same
// order each time, the verification plan (scratch runs, workgroup list) is
// made on the device, and failures are flags in a device status word -- so the
// capture holds only kernels and device-to-device copies, and a launch is one
// hipGraphLaunch with no host synchronisation.  The recorded graph bakes in
// the index's tables and the size of its cache list, so a launch after an
// update or a rebuild records the graph again first.
#include "gts_internal.h"
#include "kernels.h"

struct gts_plan {
    gts_index *idx = nullptr;
    int64_t nq = 0, cap = 0;
    gts_query_opts opts{};
    hipStream_t stream = nullptr;   // recording stream (default priority)
    hipEvent_t done = nullptr;      // recorded after each launch
    gts::DevBuf space;              // intermediate space of the recorded search
    gts::Arena arena;
    gts::QueryCtx ctx;
    gts_plan_io io{};
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    uint32_t epoch = 0;
    int64_t rebuilds = -1;
    void drop()
    {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        exec = nullptr;
        graph = nullptr;
    }
    ~gts_plan()
    {
        if (done) (void)hipEventSynchronize(done);
        drop();
        for (gts::DevBuf &w : ctx.ws) w.release();
        ctx.arena = nullptr;
        if (stream) (void)hipStreamDestroy(stream);
        if (done) (void)hipEventDestroy(done);
    }
};

namespace {

constexpr int64_t kDefaultSpace = (int64_t)1 << 30;

void record(gts_plan *p)
{
    // the last launch still reads the space and the graph about to be replaced
    GTS_HIP(hipEventSynchronize(p->done));
    p->drop();
    for (gts::DevBuf &w : p->ctx.ws) w.release();
    p->arena.used = 0;
    gts::QueryCtx &cx = p->ctx;
    cx.arena = &p->arena;
    cx.graph = true;
    cx.gstatus = reinterpret_cast<uint32_t *>(p->io.status);
    cx.timing = false;
    cx.stream = p->stream;
    const gts::IndexData &d = p->idx->data;
    gts_objects Q{};
    Q.n = p->nq;
    Q.dim = d.dim;
    Q.location = GTS_DEVICE;
    Q.vecs = p->io.queries;
    gts::NoAllocOut na{p->io.offsets, p->io.ids, p->io.dist, p->cap, nullptr};
    gts_result res{};
    GTS_HIP(hipStreamBeginCapture(p->stream, hipStreamCaptureModeThreadLocal));
    try {
        gts::k::fill_u32(cx.gstatus, 1, 0u, p->stream);
        gts::search(p->idx, &cx, &Q, p->io.radius, p->io.k, &p->opts, &res, &na);
    } catch (...) {
        hipGraph_t g = nullptr;
        (void)hipStreamEndCapture(p->stream, &g);
        if (g) (void)hipGraphDestroy(g);
        throw;
    }
    GTS_HIP(hipStreamEndCapture(p->stream, &p->graph));
    GTS_HIP(hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0));
    p->epoch = p->idx->epoch;
    p->rebuilds = p->idx->rebuilds;
}

}  // namespace

using namespace gts;

extern "C" {

gts_status gts_plan_create(gts_index *idx, int64_t nq, int64_t answer_capacity, const gts_query_opts *opts,
                           const gts_plan_io *io, gts_plan **out)
{
    return run_guarded([&] {
        GTS_CHECK(idx != nullptr && io != nullptr && out != nullptr, GTS_EINVAL, "null argument");
        GTS_CHECK(idx->data.metric == GTS_L2_F32, GTS_ENOTSUP, "search plans take vector indexes");
        GTS_CHECK(nq >= 1 && nq < ((int64_t)1 << 31), GTS_EINVAL, "a plan needs 1 .. 2^31-1 queries");
        GTS_CHECK(answer_capacity >= 0, GTS_EINVAL, "negative answer capacity");
        GTS_CHECK(!opts || opts->mode == GTS_MODE_BATCHED, GTS_EINVAL, "search plans run the batched form");
        GTS_CHECK(io->queries && io->radius && io->k && io->offsets && io->status, GTS_EINVAL,
                  "null plan buffer");
        GTS_CHECK(answer_capacity == 0 || (io->ids && io->dist), GTS_EINVAL, "null plan answer buffers");
        auto p = std::make_unique<gts_plan>();
        p->idx = idx;
        p->nq = nq;
        p->cap = answer_capacity;
        p->io = *io;
        if (opts) p->opts = *opts;
        p->opts.mode = GTS_MODE_BATCHED;
        const int64_t space = p->opts.mem_budget_bytes > 0 ? p->opts.mem_budget_bytes : kDefaultSpace;
        p->space.alloc((size_t)space);
        p->arena.base = p->space.as<uint8_t>();
        p->arena.size = (size_t)space;
        GTS_HIP(hipStreamCreateWithFlags(&p->stream, hipStreamNonBlocking));
        GTS_HIP(hipEventCreateWithFlags(&p->done, hipEventDisableTiming));
        // the pinned staging the search expects, made before recording
        GTS_CHECK(p->ctx.pinned(staging_bytes(nq)) != nullptr, GTS_ENOMEM, "pinned staging of a search plan");
        p->ctx.pin_fixed = true;
        record(p.get());
        *out = p.release();
    });
}

gts_status gts_plan_launch(gts_plan *p, void *hip_stream)
{
    return run_guarded([&] {
        GTS_CHECK(p != nullptr, GTS_EINVAL, "null plan");
        if (p->idx->epoch != p->epoch || p->idx->rebuilds != p->rebuilds) record(p);
        hipStream_t st = hip_stream ? static_cast<hipStream_t>(hip_stream) : p->idx->stream;
        GTS_HIP(hipGraphLaunch(p->exec, st));
        GTS_HIP(hipEventRecord(p->done, st));
    });
}

gts_status gts_plan_destroy(gts_plan *p)
{
    return run_guarded([&] {
        delete p;
    });
}

}  // extern "C"
