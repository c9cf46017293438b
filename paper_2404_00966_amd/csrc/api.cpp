// The C ABI of libgts.so (declared in include/gts.h): argument checks, error
// text, and the lifetime of indexes and results.  No exception crosses it.
#include <cstring>
#include <functional>
#include <string>

#include "gts_internal.h"

namespace gts {

void free_result(gts_result *r);
bool result_on_device(const gts_result *r);

[[noreturn]] void fail(gts_status s, const std::string &msg) { throw Error(s, msg); }

namespace {

thread_local std::string g_last_error;

template <class F> gts_status guarded(F &&f)
{
    try {
        f();
        g_last_error.clear();
        return GTS_OK;
    } catch (const Error &e) {
        g_last_error = e.what();
        return e.status;
    } catch (const std::bad_alloc &) {
        g_last_error = "host allocation failed";
        return GTS_ENOMEM;
    } catch (const std::exception &e) {
        g_last_error = e.what();
        return GTS_EINVAL;
    } catch (...) {
        g_last_error = "unknown failure";
        return GTS_EINVAL;
    }
}

}  // namespace

gts_status run_guarded(const std::function<void()> &f) { return guarded(f); }

}  // namespace gts

using namespace gts;

extern "C" {

const char *gts_last_error(void) { return g_last_error.c_str(); }

gts_status gts_build_index(const gts_objects *objs, int32_t metric, int32_t num_pivots, int32_t fanout,
                           const gts_build_opts *opts, void *hip_stream, gts_index **out)
{
    return guarded([&] {
        GTS_CHECK(out != nullptr, GTS_EINVAL, "null output handle");
        GTS_CHECK(objs != nullptr, GTS_EINVAL, "null objects");
        GTS_CHECK(metric == GTS_L2_F32 || metric == GTS_EDIT_U8 || metric == GTS_COSINE_F32 || metric == GTS_L1_F32,
                  GTS_EINVAL, "unknown metric");
        // the angular metric is an L2 index over unit vectors; the Manhattan
        // metric is the vector index with L1 distances
        const bool angular = metric == GTS_COSINE_F32;
        const bool l1 = metric == GTS_L1_F32;
        if (angular || l1) metric = GTS_L2_F32;
        GTS_CHECK(num_pivots >= 1 && num_pivots <= kMaxPivots, GTS_EINVAL, "num_pivots must be in [1, 32]");
        GTS_CHECK(fanout >= 2 && fanout <= 64, GTS_EINVAL, "fanout must be in [2, 64]");
        GTS_CHECK(objs->n >= 1, GTS_EINVAL, "an index needs at least one object");
        if (metric == GTS_L2_F32) GTS_CHECK(objs->dim >= 1, GTS_EINVAL, "dim must be >= 1");
        auto idx = std::make_unique<gts_index>();
        idx->stream = static_cast<hipStream_t>(hip_stream);
        idx->ctx.stream = idx->stream;
        // the no-allocation search's context: same stream, pinned staging
        // for its largest batch made now (that call allocates nothing)
        idx->ctx_na.stream = idx->stream;
        GTS_CHECK(idx->ctx_na.pinned(staging_bytes(kNoAllocMaxQueries)) != nullptr, GTS_ENOMEM,
                  "pinned staging of the no-allocation search");
        idx->ctx_na.pin_fixed = true;
        if (opts) idx->opts = *opts;
        GTS_CHECK(idx->opts.precision == GTS_PRECISION_DEFAULT || idx->opts.precision == GTS_BF16_GUARDED ||
                      idx->opts.precision == GTS_FP32,
                  GTS_EINVAL, "precision must be GTS_BF16_GUARDED or GTS_FP32");
        GTS_CHECK(idx->opts.reserved0 == 0, GTS_EINVAL, "gts_build_opts.reserved0 must be 0");
        if (idx->opts.precision == GTS_PRECISION_DEFAULT) idx->opts.precision = GTS_BF16_GUARDED;
        // the path is borrowed: keep a copy
        if (idx->opts.tune_cache) idx->tune_cache = idx->opts.tune_cache;
        idx->opts.tune_cache = nullptr;
        if (idx->opts.max_strlen <= 0 || idx->opts.max_strlen > kMaxStrlen) idx->opts.max_strlen = kMaxStrlen;
        if (idx->opts.cache_limit <= 0) idx->opts.cache_limit = 4096;
        if (idx->opts.mem_budget_bytes <= 0) {
            size_t free_b = 0, total_b = 0;
            GTS_HIP(hipMemGetInfo(&free_b, &total_b));
            idx->opts.mem_budget_bytes = (int64_t)(free_b / 4);
        }
        idx->num_pivots = num_pivots;
        idx->fanout = fanout;
        idx->data.max_strlen = idx->opts.max_strlen;
        HostObjects h;
        idx->angular = angular;
        idx->l1 = l1;
        DevBuf rows;   // vector objects given in device memory stay there
        const bool on_device = metric == GTS_L2_F32 && objs->location == GTS_DEVICE;
        GTS_CHECK(objs->n < ((int64_t)1 << 31), GTS_ENOTSUP, "at most 2^31-1 objects");
        if (on_device) {
            read_rows_device(objs, objs->dim, angular, idx->stream, &rows);
            h.metric = metric;
            h.dim = objs->dim;
            h.ids.resize(objs->n);
        } else {
            read_objects(objs, metric, metric == GTS_L2_F32 ? objs->dim : 0, idx->opts.max_strlen, &h, angular);
        }
        for (int64_t i = 0; i < h.count(); i++) h.ids[i] = (uint32_t)i;
        idx->next_id = h.count();
        idx->cache_host.metric = metric;
        idx->cache_host.dim = h.dim;
        build_tree(idx.get(), h, on_device ? &rows : nullptr);
        tune_cache_load(idx.get());
        *out = idx.release();
    });
}

gts_status gts_search(gts_index *idx, const gts_objects *Q, const float *radius, const int32_t *k,
                      const gts_query_opts *opts, gts_result *out)
{
    return guarded([&] {
        GTS_CHECK(idx != nullptr, GTS_EINVAL, "null index");
        search(idx, &idx->ctx, Q, radius, k, opts, out);
    });
}

gts_status gts_range_query(gts_index *idx, const gts_objects *Q, const float *radius, const gts_query_opts *opts,
                           gts_result *out)
{
    return guarded([&] {
        GTS_CHECK(idx != nullptr, GTS_EINVAL, "null index");
        GTS_CHECK(Q != nullptr, GTS_EINVAL, "null queries");
        GTS_CHECK(radius != nullptr || Q->n == 0, GTS_EINVAL, "null radius");
        search(idx, &idx->ctx, Q, radius, nullptr, opts, out);
    });
}

gts_status gts_knn_query(gts_index *idx, const gts_objects *Q, const int32_t *k, const gts_query_opts *opts,
                         gts_result *out)
{
    return guarded([&] {
        GTS_CHECK(idx != nullptr, GTS_EINVAL, "null index");
        GTS_CHECK(Q != nullptr, GTS_EINVAL, "null queries");
        GTS_CHECK(k != nullptr || Q->n == 0, GTS_EINVAL, "null k");
        for (int64_t i = 0; i < Q->n; i++) GTS_CHECK(k[i] >= 1, GTS_EINVAL, "k must be >= 1");
        search(idx, &idx->ctx, Q, nullptr, k, opts, out);
    });
}

gts_status gts_insert(gts_index *idx, const gts_objects *objs, int64_t *out_ids)
{
    return guarded([&] {
        GTS_CHECK(idx != nullptr, GTS_EINVAL, "null index");
        HostObjects h;
        read_objects(objs, idx->data.metric, idx->data.dim, idx->opts.max_strlen, &h, idx->angular);
        insert_objects(idx, h, out_ids);
    });
}

gts_status gts_update_batch(gts_index *idx, const gts_objects *objs, const int64_t *del_ids, int64_t n_del,
                            int64_t *out_ids, int64_t *n_deleted)
{
    return guarded([&] {
        GTS_CHECK(idx != nullptr, GTS_EINVAL, "null index");
        GTS_CHECK(n_del >= 0, GTS_EINVAL, "negative count");
        GTS_CHECK(del_ids != nullptr || n_del == 0, GTS_EINVAL, "null ids");
        HostObjects h;
        h.metric = idx->data.metric;
        h.dim = idx->data.dim;
        if (objs) read_objects(objs, idx->data.metric, idx->data.dim, idx->opts.max_strlen, &h, idx->angular);
        update_batch(idx, h, del_ids, n_del, out_ids, n_deleted);
    });
}

gts_status gts_delete(gts_index *idx, const int64_t *ids, int64_t n, int64_t *n_deleted)
{
    return guarded([&] {
        GTS_CHECK(idx != nullptr, GTS_EINVAL, "null index");
        GTS_CHECK(n >= 0, GTS_EINVAL, "negative count");
        GTS_CHECK(ids != nullptr || n == 0, GTS_EINVAL, "null ids");
        const int64_t done = delete_ids(idx, ids, n);
        if (n_deleted) *n_deleted = done;
    });
}

gts_status gts_result_copy(const gts_result *res, int32_t dst_location, int64_t *offsets, int64_t *ids, void *dist)
{
    return guarded([&] {
        GTS_CHECK(res != nullptr, GTS_EINVAL, "null result");
        GTS_CHECK(dst_location == GTS_HOST || dst_location == GTS_DEVICE, GTS_EINVAL, "bad location");
        const bool src_dev = result_on_device(res);
        hipMemcpyKind kind = src_dev ? (dst_location == GTS_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost)
                                     : (dst_location == GTS_DEVICE ? hipMemcpyHostToDevice : hipMemcpyHostToHost);
        if (offsets && res->offsets) GTS_HIP(hipMemcpy(offsets, res->offsets, (res->nq + 1) * sizeof(int64_t), kind));
        if (res->total > 0) {
            if (ids) GTS_HIP(hipMemcpy(ids, res->ids, res->total * sizeof(int64_t), kind));
            const void *src = res->dist_f32 ? (const void *)res->dist_f32 : (const void *)res->dist_i32;
            if (dist && src) GTS_HIP(hipMemcpy(dist, src, res->total * 4, kind));
        }
    });
}

gts_status gts_result_free(gts_result *res)
{
    return guarded([&] {
        if (res) free_result(res);
    });
}

gts_status gts_destroy(gts_index *idx)
{
    return guarded([&] {
        if (!idx) return;
        if (idx->stream) (void)hipStreamSynchronize(idx->stream);
        else (void)hipDeviceSynchronize();
        delete idx;
    });
}

gts_status gts_get_info(const gts_index *idx, gts_index_info *out)
{
    return guarded([&] {
        GTS_CHECK(idx != nullptr && out != nullptr, GTS_EINVAL, "null argument");
        const IndexData &d = idx->data;
        std::memset(out, 0, sizeof(*out));
        out->metric = idx->angular ? GTS_COSINE_F32 : idx->l1 ? GTS_L1_F32 : d.metric;
        out->dim = d.dim;
        out->num_pivots = d.m;
        out->fanout = d.tree.fanout;
        out->levels = d.tree.levels;
        out->max_strlen = d.max_strlen;
        out->n_indexed = d.n;
        out->n_cache = idx->cache.n_live;
        out->n_live = d.n - idx->n_deleted_tree + idx->cache.n_live;
        out->n_nodes = d.tree.n_nodes;
        out->n_leaves = d.tree.n_leaves;
        out->n_slabs = d.n_slabs;
        out->rebuilds = idx->rebuilds;
        int64_t bytes = 0;
        for (const DevBuf *b : {&d.X32, &d.X16t, &d.xn, &d.xe, &d.P32, &d.PT, &d.slab_emax, &d.slab_nmax,
                                &d.slab_leaf_lo, &d.slab_leaf_hi, &d.chars, &d.soff, &d.PTe, &d.PTa, &d.pchars,
                                &d.poff, &d.ids, &d.tomb, &d.del_ep, &d.tree.box_aos, &d.tree.box_lo, &d.tree.box_hi,
                                &d.tree.leaf_first, &d.tree.leaf_cnt})
            bytes += (int64_t)b->bytes;
        out->device_bytes = bytes;
        out->rebuild_ms = idx->rebuild_ms;
        out->epoch = idx->epoch;
    });
}

gts_status gts_get_stats(const gts_index *idx, gts_stats *out)
{
    return guarded([&] {
        GTS_CHECK(idx != nullptr && out != nullptr, GTS_EINVAL, "null argument");
        *out = idx->ctx.stats;
    });
}

gts_status gts_set_timing(gts_index *idx, int32_t enable)
{
    return guarded([&] {
        GTS_CHECK(idx != nullptr, GTS_EINVAL, "null index");
        idx->ctx.timing = enable != 0;
    });
}

}  // extern "C"
