// Query orchestration: one call runs a mixed batch of range and kNN queries
// through the GPU stages, under the two-stage memory budget of Sec. 5.1.
//
//   prep     query -> pivot distances (Lemma 1 needs d(q, p) for every pivot),
//            bf16 query fragments / match tables
//   bound    kNN: an upper bound of the k-th distance (Sec. 5.2: kNN answered
//            as a range query once that distance is bounded)
//   nodes    layer-by-layer child test of every (query tile, node)
//   cands    L2: bf16 MFMA distances over surviving (slab, tile) pairs;
//            EDIT: Lemma 1 on every object of every surviving (leaf, tile)
//   group    candidates grouped by query
//   verify   exact distances, per-query selection, (distance, id) order
//   output   CSR assembly
//
// When one batch's candidates would not fit the budget, the queries are split
// into groups of whole 16-query blocks processed one after another (the
// "second stage"); answers do not depend on the grouping.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>

#include "gts_internal.h"
#include "kernels.h"

namespace gts {

namespace {

enum Ws {
    W_Q32, W_Q16, W_QN, W_QE, W_QP, W_BASE, W_T, W_THR, W_KQ, W_HOME, W_QCHARS, W_QOFF, W_PEQ, W_QLEN,
    W_MASK, W_ITEMS, W_SMALL, W_CANDS, W_GROUPED, W_QCOUNT, W_QOFF64, W_OUTKEYS, W_OUTCNT, W_RESOFF, W_SCRATCH,
    W_FRONTIER, W_BIGOFF, W_CURSOR, W_COUNTERS, W_RES_IDS, W_RES_DIST, W_RES_OFF, W_NEAR, W_TMP, W_PERM,
    W_TMP2, W_RES_IDS2, W_RES_DIST2, W_OFF_ORIG, W_CUT, W_TQE, W_QCELLS0, W_QCNT0, W_QCELLS, W_QCNT, W_ORDER, W_PAIR_TILE, W_PAIR_MASK, W_SWEEP_ITEMS, W_BLKQ,
    W_SORT_TMP, W_HOME2, W_PBASE, W_PKQ, W_PQP, W_PQ32, W_PNEAR, W_PIV, W_POSOF, W_HOMEC, W_PLEN, W_POFF, W_PCHARS,
    W_BADQ, W_QEP, W_PQEP, W_TMIN, W_TMAX, W_TILEW, W_VNEED, W_VFLAG, W_VNOFF, W_NBLK, W_VCUR, W_COUNT
};
static_assert(W_COUNT <= kWorkspaceSlots, "too few workspace slots in QueryCtx");

struct ResultPriv {
    void *offsets = nullptr, *ids = nullptr, *dist = nullptr;
    bool device = false;
};

}  // namespace

void free_result(gts_result *r);

namespace {

template <class T> T *wsp(QueryCtx *cx, int slot, size_t count)
{
    const size_t need = std::max<size_t>(count * sizeof(T), 64);
    DevBuf &b = cx->ws[slot];
    if (cx->arena) {
        // no-allocation search: a view carved from the arena
        if (!b.p || b.bytes < need) {
            b.release();
            b.p = cx->arena->take(need);
            b.bytes = need;
            b.owned = false;
        }
        return b.as<T>();
    }
    b.alloc(need);
    return b.as<T>();
}

// Small device counters (32-bit words): [0, 1] the 64-bit candidate count,
// [2] the edit leaf-item count, [4, 7) the sweep's work-list counts
constexpr int kSmallWords = 16;
constexpr int kSmallItems = 2;
constexpr int kSmallSweep = 4;

// Pinned host staging of one search call: device-to-host the permutation
// (nq int32), the small counters, the group's segment offsets, counts and
// the statistics counters; host-to-device the workgroup-mode query list, the
// scratch offsets and the result offsets, and (edit distance) the query
// offsets, lengths, length order and positions in it.  Regions are disjoint,
// so no host write waits for an earlier copy.
struct PinLayout {
    size_t perm = 0, small = 0, qoff = 0, counts = 0, counters = 0, blk = 0, big = 0, offs = 0;
    size_t in_off = 0, in_len = 0, in_ord = 0, in_pos = 0, bytes = 0;
    explicit PinLayout(int64_t nq)
    {
        auto up = [](size_t v) { return (v + 255) / 256 * 256; };
        small = up((size_t)nq * sizeof(int32_t));
        qoff = small + 256;
        counts = up(qoff + (size_t)(nq + 1) * sizeof(int64_t));
        counters = up(counts + (size_t)(nq + 1) * sizeof(uint32_t));
        blk = up(counters + (size_t)k::kCounterWords * sizeof(uint64_t));   // host-to-device: workgroup-mode queries
        big = up(blk + (size_t)(nq + 1) * sizeof(int32_t));    // scratch offsets
        offs = up(big + (size_t)(nq + 1) * sizeof(int64_t));   // result offsets
        in_off = up(offs + (size_t)(nq + 1) * sizeof(int64_t));
        in_len = up(in_off + (size_t)(nq + 1) * sizeof(int64_t));
        in_ord = up(in_len + (size_t)nq * sizeof(int32_t));
        in_pos = up(in_ord + (size_t)nq * sizeof(int32_t));
        bytes = up(in_pos + (size_t)nq * sizeof(int32_t));
    }
};

// Result storage: offsets, ids and distances in one allocation (freed here
// unless released to a result).
struct ResultMem {
    void *p = nullptr;
    bool device = false;
    size_t id_at = 0, dist_at = 0, bytes = 0;
    int64_t cap = 0;                // ids / distances it holds
    ResultMem() = default;
    ResultMem(const ResultMem &) = delete;
    ResultMem &operator=(const ResultMem &) = delete;
    ResultMem(ResultMem &&o) noexcept { *this = std::move(o); }
    ResultMem &operator=(ResultMem &&o) noexcept
    {
        if (this != &o) {
            reset();
            p = o.p;
            device = o.device;
            id_at = o.id_at;
            dist_at = o.dist_at;
            bytes = o.bytes;
            cap = o.cap;
            o.p = nullptr;
        }
        return *this;
    }
    void *release()
    {
        void *r = p;
        p = nullptr;
        return r;
    }
    void reset()
    {
        if (p) (void)(device ? hipFree(p) : hipHostFree(p));
        p = nullptr;
    }
    ~ResultMem() { reset(); }
};

ResultMem result_alloc(int64_t nq, int64_t entries, bool device)
{
    ResultMem m;
    m.device = device;
    const size_t off_bytes = (nq + 1) * sizeof(int64_t);
    m.cap = std::max<int64_t>(entries, 1);
    m.id_at = (off_bytes + 255) / 256 * 256;
    m.dist_at = m.id_at + ((size_t)m.cap * sizeof(int64_t) + 255) / 256 * 256;
    m.bytes = m.dist_at + (size_t)m.cap * sizeof(float);
    const hipError_t e = device ? hipMalloc(&m.p, m.bytes) : hipHostMalloc(&m.p, m.bytes, hipHostMallocDefault);
    if (e != hipSuccess) m.p = nullptr;
    return m;
}

struct GroupOut {
    std::vector<uint32_t> counts;  // per query of the group
    DevBuf ids, dist;              // CSR pieces of the group (unless direct)
    int64_t total = 0;
    bool direct = false;           // sorted keys left in the workspace (W_OUTKEYS, W_QOFF64, W_OUTCNT)
    ResultMem pre;                 // direct: result storage for every candidate, allocated while verify runs
    // a group whose candidates overflowed: how many it produced, and the
    // (query, object) pairs of each of its query tiles (empty: unknown)
    uint64_t attempts = 0;
    std::vector<unsigned long long> tile_work;
};

double now_ms()
{
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

}  // namespace

// ---------------------------------------------------------------------------
// Reading user objects (host or device) into host memory, with validation.
// ---------------------------------------------------------------------------
void read_objects(const gts_objects *o, int32_t metric, int32_t dim, int32_t max_strlen, HostObjects *out,
                  bool angular)
{
    GTS_CHECK(o != nullptr, GTS_EINVAL, "null object set");
    GTS_CHECK(o->n >= 0, GTS_EINVAL, "negative object count");
    GTS_CHECK(o->location == GTS_HOST || o->location == GTS_DEVICE, GTS_EINVAL, "bad location");
    const hipMemcpyKind kind = o->location == GTS_DEVICE ? hipMemcpyDeviceToHost : hipMemcpyHostToHost;
    out->metric = metric;
    out->dim = dim;
    out->clear();
    const int64_t n = o->n;
    if (metric == GTS_L2_F32) {
        GTS_CHECK(o->dim == dim, GTS_EINVAL, "dimension mismatch");
        if (n == 0) return;
        GTS_CHECK(o->vecs != nullptr, GTS_EINVAL, "null vectors");
        out->vecs.resize((size_t)n * dim);
        GTS_HIP(hipMemcpy(out->vecs.data(), o->vecs, out->vecs.size() * sizeof(float), kind));
        for (float v : out->vecs) GTS_CHECK(std::isfinite(v), GTS_EINVAL, "non-finite vector value");
        if (angular)
            for (int64_t i = 0; i < n; i++) {
                float *x = out->vecs.data() + (size_t)i * dim;
                double s = 0.0;
                for (int j = 0; j < dim; j++) s += (double)x[j] * (double)x[j];
                const double nrm = std::sqrt(s);
                GTS_CHECK(nrm > 0.0 && std::isfinite(nrm), GTS_EINVAL, "a zero vector has no direction (angular metric)");
                for (int j = 0; j < dim; j++) x[j] = (float)((double)x[j] / nrm);
            }
    } else {
        if (n == 0) return;
        GTS_CHECK(o->offsets != nullptr, GTS_EINVAL, "null string offsets");
        out->offsets.resize(n + 1);
        GTS_HIP(hipMemcpy(out->offsets.data(), o->offsets, (n + 1) * sizeof(int64_t), kind));
        GTS_CHECK(out->offsets[0] == 0, GTS_EINVAL, "offsets[0] must be 0");
        for (int64_t i = 0; i < n; i++) {
            const int64_t len = out->offsets[i + 1] - out->offsets[i];
            GTS_CHECK(len >= 0, GTS_EINVAL, "offsets must be non-decreasing");
            GTS_CHECK(len <= max_strlen, GTS_EINVAL,
                      "string of length " + std::to_string(len) + " exceeds max_strlen " + std::to_string(max_strlen));
        }
        const int64_t total = out->offsets[n];
        out->chars.resize(total);
        if (total) {
            GTS_CHECK(o->chars != nullptr, GTS_EINVAL, "null string bytes");
            GTS_HIP(hipMemcpy(out->chars.data(), o->chars, total, kind));
        }
    }
    out->ids.resize(n);
}

void read_rows_device(const gts_objects *o, int32_t dim, bool angular, hipStream_t st, DevBuf *rows)
{
    GTS_CHECK(o != nullptr && o->location == GTS_DEVICE, GTS_EINVAL, "device rows expected");
    GTS_CHECK(o->dim == dim && dim >= 1, GTS_EINVAL, "dimension mismatch");
    const int64_t n = o->n;
    GTS_CHECK(n >= 1 && o->vecs != nullptr, GTS_EINVAL, "null vectors");
    const int dp = (dim + 3) / 4 * 4;
    rows->alloc((size_t)n * dp * sizeof(float));
    rows_to_device(rows->as<float>(), dp, o->vecs, dim, n, true, st);
    DevBuf flags;
    flags.alloc(2 * sizeof(uint32_t));
    k::fill_u32(flags.as<uint32_t>(), 2, 0u, st);
    k::check_finite(rows->as<float>(), n, dim, dp, flags.as<uint32_t>(), st);
    if (angular) k::normalize_rows(rows->as<float>(), n, dim, dp, flags.as<uint32_t>() + 1, st);
    uint32_t h[2] = {0u, 0u};
    GTS_HIP(hipMemcpyAsync(h, flags.p, sizeof(h), hipMemcpyDeviceToHost, st));
    GTS_HIP(hipStreamSynchronize(st));
    GTS_CHECK(h[0] == 0, GTS_EINVAL, "non-finite vector value");
    GTS_CHECK(h[1] == 0, GTS_EINVAL, "a zero vector has no direction (angular metric)");
}

namespace k {
void require(bool ok, const char *what)
{
    if (!ok) fail(GTS_ENOTSUP, what);
}

void check_launch(const char *name)
{
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) fail(GTS_EDEVICE, std::string("kernel launch failed in ") + name + ": " + hipGetErrorString(e));
}
}  // namespace k

// ---------------------------------------------------------------------------
// One query group [q0, q0 + ng): candidates -> verified, sorted answers.
// Returns false when the candidates overflow `cap` (nothing produced).
// ---------------------------------------------------------------------------
namespace {

struct Batch {
    int64_t nq = 0;
    bool any_knn = false;
    int mode = GTS_MODE_BATCHED;
    int max_qlen = 0;          // longest query string (EDIT)
    float max_radius = 0.f;    // largest range radius
    int64_t ntiles_all = 0;    // query tiles of the whole batch
    int precision = GTS_BF16_GUARDED;   // L2 candidate selection (batched form)
    int sweep_grid_per_cu = 2;          // MFMA sweep workgroups per CU (tuned)
    bool check_bound = false;           // count bf16 interval violations
    bool no_prune = false;              // L2 control: every (leaf, query) pair kept
    bool check_q = false;               // the query rows were checked on the device (flag in W_BADQ)
    // what the batch sees (server batches: see SnapView)
    const uint32_t *tomb_prod = nullptr;    // tombstones of the candidate producers
    const uint32_t *tomb_bound = nullptr;   // tombstones of the kNN bounds
    const uint32_t *qep = nullptr;          // [nq] admission epochs (null: all at e_now)
    uint32_t e_now = 0;
    int64_t cache_count = 0;                // cache slots to scan
};

void rec(QueryCtx *cx, int i)
{
    if (cx->timing) GTS_HIP(hipEventRecord(cx->ev[i], cx->stream));
}

bool run_group(gts_index *idx, QueryCtx *cx, const Batch &b, int64_t q0, int64_t ng, int64_t cap, bool direct,
               bool result_on_device, uint8_t *pin, const PinLayout &pl, GroupOut *go, double *stage_ms)
{
    hipStream_t st = cx->stream;
    IndexData &d = idx->data;
    Tree &t = d.tree;
    const bool l2 = d.metric == GTS_L2_F32;
    const int mpad = t.mpad;
    k::TreeView tv{t.box_aos.as<float>(), t.box_lo.as<float>(), t.box_hi.as<float>(), t.leaf_first.as<int32_t>(),
                   t.leaf_cnt.as<int32_t>(), t.n_nodes, t.n_leaves, t.leaf0, t.fanout, t.levels, mpad};
    k::L2View ov{d.X32.as<float>(), d.xn.as<float>(), d.xe.as<float>(), d.X16t.as<uint16_t>(), d.n, d.npad,
                 d.dim, d.dp, d.ksteps};
    k::EditView oe{d.chars.as<uint8_t>(), d.soff.as<int32_t>(), d.n, idx->lut.as<uint8_t>(), idx->arows};
    const int ntiles = (int)((ng + kQTile - 1) / kQTile);

    float *QP = cx->ws[W_QP].as<float>() + q0 * mpad;
    float *base = cx->ws[W_BASE].as<float>() + q0;
    float *T = cx->ws[W_T].as<float>() + q0;
    float *thr = cx->ws[W_THR].as<float>() + q0;
    int32_t *kq = cx->ws[W_KQ].as<int32_t>() + q0;
    k::QueryL2 qv{};
    k::QueryEdit qe{};
    if (l2) {
        qv.Q32 = cx->ws[W_Q32].as<float>() + q0 * d.dp;
        qv.Q16t = cx->ws[W_Q16].as<uint16_t>() + q0 * d.ksteps * 32;
        qv.qn = cx->ws[W_QN].as<float>() + q0;
        qv.qe = cx->ws[W_QE].as<float>() + q0;
    } else {
        qe.chars = cx->ws[W_QCHARS].as<uint8_t>();
        qe.off = cx->ws[W_QOFF].as<int64_t>() + q0;
        qe.peq = cx->ws[W_PEQ].as<uint64_t>() + q0 * idx->arows * 4;
    }
    uint32_t *small = wsp<uint32_t>(cx, W_SMALL, kSmallWords);
    unsigned long long *counters = cx->ws[W_COUNTERS].as<unsigned long long>();
    k::fill_u32(small, kSmallWords, 0u, st);
    k::CandCount *ccount = reinterpret_cast<k::CandCount *>(small);
    k::Cand *cands = wsp<k::Cand>(cx, W_CANDS, cap);
    const uint32_t *tomb = b.tomb_prod;
    const uint32_t *qep = b.qep ? b.qep + q0 : nullptr;
    const uint32_t *del_ep = b.qep ? d.del_ep.as<uint32_t>() : nullptr;

    const bool plain = b.mode == GTS_MODE_PLAIN || (l2 && d.dim > kMaxMfmaDim);
    // float32 selection: Lemma 1 on the pivot table instead of bf16 tiles
    // (the Manhattan metric always selects on the float32 pivot table)
    const bool sel32 = l2 && !plain && (b.precision == GTS_FP32 || idx->l1);
    int64_t n_wide = 0;
    rec(cx, 2);
    if (plain) {
        const int grid = (int)std::min<int64_t>(ng, 1024);
        k::PlainArgs pa{};
        pa.nq = ng;
        pa.base = base;
        pa.kq = kq;
        pa.frontier = wsp<int32_t>(cx, W_FRONTIER, (size_t)grid * 2 * t.n_leaves);
        pa.grid = grid;
        pa.tomb = tomb;
        pa.ids = d.ids.as<uint32_t>();
        pa.out = cands;
        pa.out_count = ccount;
        pa.out_cap = cap;
        pa.counters = counters;
        pa.delta = (float)((d.dim + 8) * 5.9604645e-8);
        pa.pt_max = d.pt_max;
        pa.leaf_piv32 = l2 && d.lpad > 0 ? d.PL32.as<float>() : nullptr;
        pa.leafR = l2 && d.lpad > 0 ? d.leafR.as<float>() : nullptr;
        pa.angular = idx->angular ? 1 : 0;
        pa.l1 = idx->l1 ? 1 : 0;
        rec(cx, 3);
        if (l2) k::plain_l2(tv, ov, d.P32.as<float>(), d.m, d.PT.as<float>(), qv.Q32, pa, st);
        else k::plain_edit(tv, oe, d.pchars.as<uint8_t>(), d.poff.as<int32_t>(), d.m, d.PTe.as<uint8_t>(), qe, pa, st);
        rec(cx, 4);
    } else {
        uint64_t *mask = wsp<uint64_t>(cx, W_MASK, (size_t)t.n_leaves * ntiles);
        int32_t *items = nullptr;
        const int64_t item_cap = t.n_leaves * ntiles;
        if (l2 && b.no_prune) {
            k::fill_u32(reinterpret_cast<uint32_t *>(mask), (int64_t)2 * t.n_leaves * ntiles, 0xffffffffu, st);
        } else if (l2) {
            k::leaf_box(tv, QP, thr, ng, ntiles, mask, counters, st);
        } else {
            // leaves of the cells that passed (cell masks of the whole batch,
            // this group's tiles from column q0 / 64), then the item list
            items = wsp<int32_t>(cx, W_ITEMS, (size_t)item_cap * 2);
            const int32_t *qlen = cx->ws[W_QLEN].as<int32_t>() + q0;
            k::edit_leaf_ball(oe, qe, qlen, t.leaf_first.as<int32_t>(), d.leafR.as<float>(), d.leaf_cell.as<int32_t>(),
                              d.cell_leaf.as<int32_t>(), d.n_centres,
                              cx->ws[W_QCELLS].as<int32_t>() + q0 * k::kQueryCells, cx->ws[W_QCNT].as<int32_t>() + q0,
                              T, ng, ntiles, b.max_qlen, mask, items, small + kSmallItems, item_cap, t.n_leaves, st);
        }
        if (l2 && d.lpad > 0 && !b.no_prune && !idx->l1)
            k::leaf_ball(d.PL16t.as<uint16_t>(), d.pln.as<float>(), d.ple.as<float>(), d.leafR.as<float>(), t.n_leaves,
                         d.ksteps, qv.Q16t, qv.qn, qv.qe, T, ng, ntiles, mask, t.leaf_cnt.as<int32_t>(), counters, st);
        k::SlabView sv{d.slab_emax.as<float>(), d.slab_nmax.as<float>(), d.slab_leaf_lo.as<int32_t>(),
                       d.slab_leaf_hi.as<int32_t>(), d.n_slabs};
        k::SweepWork sw{};
        if (sel32) {
            // the (leaf, tile) work list of the float32 object filter
            items = wsp<int32_t>(cx, W_ITEMS, (size_t)item_cap * 2);
            k::mask_items(mask, t.n_leaves, ntiles, items, small + kSmallItems, item_cap, st);
        } else if (l2) {
            // the sweep's work list (timed with the node stage, so that the
            // candidate stage is the MFMA sweep alone)
            const int64_t pairs = d.n_slabs * ntiles;
            const int64_t nitems = d.n_slabs * ((ntiles + k::kSweepItemTiles - 1) / k::kSweepItemTiles);
            sw = k::SweepWork{wsp<int32_t>(cx, W_PAIR_TILE, pairs), wsp<uint64_t>(cx, W_PAIR_MASK, pairs),
                              wsp<int4>(cx, W_SWEEP_ITEMS, nitems), small + kSmallSweep};
            k::slab_items(sv, mask, ntiles, sw, st);
        }
        rec(cx, 3);
        if (sel32) {
            k::l2_objfilter(tv, items, small + kSmallItems, item_cap, mask, ntiles, QP, thr, ng, d.PT.as<float>(), d.n,
                            tomb, cands, ccount, cap, counters, st);
        } else if (l2) {
            int dev = 0, cus = 256;
            GTS_HIP(hipGetDevice(&dev));
            GTS_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
            const float *tqe = cx->ws[W_TQE].as<float>() + q0;
            k::mfma_sweep(ov, sv, qv, tqe, ng, ntiles, tomb, sw, cands, ccount, cap, counters,
                          cus * b.sweep_grid_per_cu, st);
        } else {
            int32_t *qlen = cx->ws[W_QLEN].as<int32_t>() + q0;
            k::edit_objfilter(tv, items, small + kSmallItems, item_cap, mask, ntiles, QP, thr, qlen, ng, d.PTa.as<uint8_t>(),
                              d.soff.as<int32_t>(), tomb, cands, ccount, cap, counters, st);
        }
        rec(cx, 4);
    }
    // cache list: brute force, already verified
    const CacheList &c = idx->cache;
    if (b.cache_count > 0) {
        k::CacheScan cs{c.ids.as<uint32_t>(), c.ins_ep.as<uint32_t>(), c.del_ep.as<uint32_t>(),
                        l2 ? nullptr : c.cp.as<float>(), b.cache_count, d.m, mpad, qep, b.e_now, QP};
        if (l2) {
            // emission cutoff: radius (range) or the widened bound T (kNN)
            float *cut = cx->ws[W_CUT].as<float>() + q0;
            k::cache_scan_l2(qv.Q32, ng, d.dp, c.X32.as<float>(), cs, cut, cands, ccount, cap, idx->angular, st,
                             idx->l1);
        } else {
            k::cache_scan_edit(qe, oe, ng, c.chars.as<uint8_t>(), kMaxStrlen, c.slen.as<int32_t>(), cs, base, cands,
                               ccount, cap, st);
        }
    }
    // ---- group by query ----------------------------------------------------
    // No host round trip before the grouping: the scatter writes at most the
    // grouped buffer's current capacity, and a larger candidate count (known
    // at the next synchronisation) grows it and scatters again.
    uint32_t *qcount = wsp<uint32_t>(cx, W_QCOUNT, ng + 1);
    uint32_t *cursor = wsp<uint32_t>(cx, W_CURSOR, ng + 1);
    int64_t *qoff = wsp<int64_t>(cx, W_QOFF64, ng + 1);
    k::fill_u32(qcount, ng, 0u, st);
    k::fill_u32(cursor, ng, 0u, st);
    k::group_hist(cands, ccount, cap, qcount, del_ep, qep, st);
    k::scan_u32(qcount, ng, qoff, st);
    // (no-allocation search: sized for every candidate the group may keep)
    int64_t gcap = cx->arena ? cap
                             : std::max<int64_t>((int64_t)(cx->ws[W_GROUPED].bytes / sizeof(k::Cand)),
                                                 std::min<int64_t>(cap, (int64_t)1 << 20));
    k::Cand *grouped = wsp<k::Cand>(cx, W_GROUPED, gcap);
    k::group_scatter(cands, ccount, cap, qoff, cursor, grouped, gcap, del_ep, qep, st);
    rec(cx, 5);
    if (cx->graph) {
        // no host reads: fixed capacities, the verification plan made on the
        // device, the candidate overflow a status flag
        GTS_CHECK(l2 && !plain, GTS_ENOTSUP, "search plans run the batched vector form");
        k::plan_status(cx->gstatus, nullptr, ccount, cap, nullptr, 0, st);
        int64_t *big_off = wsp<int64_t>(cx, W_BIGOFF, ng + 1);
        uint64_t *scratch = wsp<uint64_t>(cx, W_SCRATCH, 2 * cap);
        int32_t *dord = wsp<int32_t>(cx, W_BLKQ, ng + 1);
        int32_t *nblk = wsp<int32_t>(cx, W_NBLK, 1);
        uint32_t *vneed = wsp<uint32_t>(cx, W_VNEED, ng + 1), *vcls = wsp<uint32_t>(cx, W_VFLAG, k::kVerifyPlanWords);
        int64_t *vnoff = wsp<int64_t>(cx, W_VNOFF, ng + 1);
        k::verify_plan_count(qoff, ng, kSortCapL2, vneed, vnoff, vcls, st);
        k::verify_plan_lists(qoff, ng, vneed, vnoff, vcls, big_off, dord, nblk, st);
        uint64_t *out_keys = wsp<uint64_t>(cx, W_OUTKEYS, std::max<int64_t>(cap, 1));
        uint32_t *out_count = wsp<uint32_t>(cx, W_OUTCNT, ng + 1);
        k::VerifyArgs va{grouped, qoff, big_off, scratch, kq, base, d.ids.as<uint32_t>(), ng, out_keys, out_count,
                         counters, idx->angular ? 1 : 0};
        uint32_t *vcur = wsp<uint32_t>(cx, W_VCUR, k::kVerifyCursorWords);
        k::fill_u32(vcur, k::kVerifyCursorWords, 0u, st);
        k::verify_l2(va, ov, qv, (float)((d.dim + 8) * 5.9604645e-8), dord, 0, !sel32, b.check_bound, st, idx->l1,
                     nblk, vcur);
        go->direct = direct;
        go->total = -1;
        return true;
    }
    uint32_t *h_small = reinterpret_cast<uint32_t *>(pin + pl.small);
    int64_t *h_qoff_pin = reinterpret_cast<int64_t *>(pin + pl.qoff);
    GTS_HIP(hipMemcpyAsync(h_small, small, kSmallWords * sizeof(uint32_t), hipMemcpyDeviceToHost, st));
    uint32_t *h_bad = h_small + 32;   // (the small-counter region of the staging holds 64 words)
    *h_bad = 0;
    if (b.check_q) GTS_HIP(hipMemcpyAsync(h_bad, cx->ws[W_BADQ].p, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
    // L2: the verification plan's counts on the device (scratch needs, class
    // sizes, the largest candidate set), read with the candidate count; the
    // edit path plans on the host from the segment offsets
    uint32_t *vneed = nullptr, *vcls = nullptr;
    int64_t *vnoff = nullptr;
    uint32_t *h_vcls = h_small + 40;           // kVerifyPlanWords words of the staging's small region
    int64_t *h_vneed = reinterpret_cast<int64_t *>(h_small + 56);
    if (l2) {
        vneed = wsp<uint32_t>(cx, W_VNEED, ng + 1);
        vcls = wsp<uint32_t>(cx, W_VFLAG, k::kVerifyPlanWords);
        vnoff = wsp<int64_t>(cx, W_VNOFF, ng + 1);
        k::verify_plan_count(qoff, ng, kSortCapL2, vneed, vnoff, vcls, st);
        GTS_HIP(hipMemcpyAsync(h_vcls, vcls, k::kVerifyPlanWords * sizeof(uint32_t), hipMemcpyDeviceToHost, st));
        GTS_HIP(hipMemcpyAsync(h_vneed, vnoff + ng, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    } else {
        GTS_HIP(hipMemcpyAsync(h_qoff_pin, qoff, (ng + 1) * sizeof(int64_t), hipMemcpyDeviceToHost, st));
    }
    GTS_HIP(hipStreamSynchronize(st));
    GTS_CHECK(*h_bad == 0, GTS_EINVAL,
              idx->angular ? "a query vector is zero or non-finite: it has no direction (angular metric)"
                           : "non-finite query value");
    const uint64_t ncand_all = *reinterpret_cast<const uint64_t *>(h_small);
    if (ncand_all > (uint64_t)cap) {
        // too many candidates for the budget: report the attempt and each
        // tile's share of the work, which sizes the smaller groups
        go->attempts = ncand_all;
        if (!plain) {
            unsigned long long *tw = wsp<unsigned long long>(cx, W_TILEW, ntiles);
            k::fill_u32(reinterpret_cast<uint32_t *>(tw), 2 * (int64_t)ntiles, 0u, st);
            k::tile_pairs(cx->ws[W_MASK].as<uint64_t>(), t.n_leaves, ntiles, t.leaf_cnt.as<int32_t>(), tw, st);
            go->tile_work.resize(ntiles);
            GTS_HIP(hipMemcpyAsync(go->tile_work.data(), tw, (size_t)ntiles * sizeof(unsigned long long),
                                   hipMemcpyDeviceToHost, st));
            GTS_HIP(hipStreamSynchronize(st));
        }
        return false;
    }
    const int64_t ncand = (int64_t)ncand_all;
    if (!plain && (!l2 || sel32) && (int64_t)h_small[kSmallItems] > t.n_leaves * ntiles)
        fail(GTS_EDEVICE, "item list overflow");
    cx->stats.candidates += ncand;
    cx->stats.leaf_pairs += plain || l2 ? 0 : (int64_t)h_small[kSmallItems];
    const int64_t *h_qoff = h_qoff_pin;   // read in place (no fresh host pages per call)
    if (ncand > gcap) {
        grouped = wsp<k::Cand>(cx, W_GROUPED, ncand);
        k::fill_u32(cursor, ng, 0u, st);
        k::group_scatter(cands, ccount, cap, qoff, cursor, grouped, ncand, del_ep, qep, st);
    }
    // segments too long for LDS sort in power-of-two scratch runs (L2: the
    // offsets, the verification order and its workgroup count made on the
    // device from the counts above; edit: on the host, into the pinned
    // staging)
    int64_t n_blk = 0;
    int64_t *big_off = nullptr;
    uint64_t *scratch = nullptr;
    int32_t *dord = nullptr;
    if (l2) {
        n_blk = (int64_t)h_vcls[0];
        cx->stats.max_query_candidates = std::max<int64_t>(cx->stats.max_query_candidates, h_vcls[2 * k::kVerifyClasses]);
        const int64_t need = *h_vneed;
        big_off = wsp<int64_t>(cx, W_BIGOFF, ng + 1);
        if (need > 0) scratch = wsp<uint64_t>(cx, W_SCRATCH, need);
        dord = wsp<int32_t>(cx, W_BLKQ, ng + 1);
        k::verify_plan_lists(qoff, ng, vneed, vnoff, vcls, big_off, dord, nullptr, st);
    } else {
        const int64_t *h_qoff = h_qoff_pin;   // read in place (no fresh host pages per call)
        int64_t *big = reinterpret_cast<int64_t *>(pin + pl.big);
        int64_t scratch_words = 0;
        bool any_big = false;
        for (int64_t q = 0; q < ng; q++) {
            const int64_t ns = h_qoff[q + 1] - h_qoff[q];
            cx->stats.max_query_candidates = std::max(cx->stats.max_query_candidates, ns);
            big[q] = -1;
            if (ns > kSortCap) {
                n_wide++;
                int64_t p = 1;
                while (p < ns) p <<= 1;
                big[q] = scratch_words;
                scratch_words += p;
                any_big = true;
            }
        }
        if (any_big) {
            big_off = wsp<int64_t>(cx, W_BIGOFF, ng);
            GTS_HIP(hipMemcpyAsync(big_off, big, ng * sizeof(int64_t), hipMemcpyHostToDevice, st));
            scratch = wsp<uint64_t>(cx, W_SCRATCH, scratch_words);
        }
    }

    // ---- verify, select, order ------------------------------------------------
    uint64_t *out_keys = wsp<uint64_t>(cx, W_OUTKEYS, std::max<int64_t>(ncand, 1));
    uint32_t *out_count = wsp<uint32_t>(cx, W_OUTCNT, ng + 1);
    k::VerifyArgs va{grouped, qoff, big_off, scratch, kq, base, d.ids.as<uint32_t>(), ng, out_keys, out_count, counters,
                     idx->angular ? 1 : 0};
    if (l2) n_wide += n_blk;
    cx->stats.wide_queries += n_wide;
    // (the verification stage's clock starts here: the planning above,
    // between the grouping and this launch, counts to the grouping)
    rec(cx, 8);
    if (l2) {
        uint32_t *vcur = wsp<uint32_t>(cx, W_VCUR, k::kVerifyCursorWords);
        k::fill_u32(vcur, k::kVerifyCursorWords, 0u, st);
        k::verify_l2(va, ov, qv, (float)((d.dim + 8) * 5.9604645e-8), dord, (int)n_blk, !plain && !sel32,
                     b.check_bound, st, idx->l1, nullptr, vcur);
    } else {
        k::verify_edit(va, oe, qe, !b.any_knn && b.max_radius <= 63.f, st);
    }
    rec(cx, 6);
    // the host waits for verify next: allocate the result meanwhile, sized for
    // every candidate (an upper bound of the answers) unless that is large
    if (direct && !cx->arena && ncand * (int64_t)(sizeof(int64_t) + sizeof(float)) <= ((int64_t)256 << 20))
        go->pre = result_alloc(b.nq, ncand, result_on_device);

    // ---- counts of this group; its CSR piece unless the keys stay -----------
    go->direct = direct;
    if (cx->arena) {
        // no-allocation search: the caller's buffers take the result on the device
        go->total = -1;
    } else if (direct && go->pre.p && result_on_device) {
        // the whole result is assembled on the device: no counts to the host
        go->total = -1;
    } else {
        uint32_t *h_counts = reinterpret_cast<uint32_t *>(pin + pl.counts);
        GTS_HIP(hipMemcpyAsync(h_counts, out_count, ng * sizeof(uint32_t), hipMemcpyDeviceToHost, st));
        GTS_HIP(hipStreamSynchronize(st));
        go->counts.assign(h_counts, h_counts + ng);
        int64_t total = 0;
        for (int64_t q = 0; q < ng; q++) total += h_counts[q];
        go->total = total;
    }
    const int64_t total = go->total;
    if (!direct) {
        int64_t *res_off = wsp<int64_t>(cx, W_RESOFF, ng + 1);
        k::scan_u32(out_count, ng, res_off, st);
        go->ids.alloc(std::max<int64_t>(total, 1) * sizeof(int64_t));
        go->dist.alloc(std::max<int64_t>(total, 1) * sizeof(float));
        k::csr_write(out_keys, qoff, out_count, res_off, ng, l2 ? 0 : 1, go->ids.as<int64_t>(),
                     go->dist.as<float>(), go->dist.as<int32_t>(), st);
    }
    rec(cx, 7);
    if (cx->timing) GTS_HIP(hipStreamSynchronize(st));
    if (cx->timing) {
        // (event 8 marks the verification launch, after the host's planning)
        const int from[] = {2, 3, 4, 8, 6}, to[] = {3, 4, 8, 6, 7};
        const int stage[] = {GTS_STAGE_NODES, plain ? GTS_STAGE_PLAIN : GTS_STAGE_CANDS, GTS_STAGE_GROUP,
                             GTS_STAGE_VERIFY, GTS_STAGE_OUTPUT};
        for (int i = 0; i < 5; i++) {
            float ms;
            GTS_HIP(hipEventElapsedTime(&ms, cx->ev[from[i]], cx->ev[to[i]]));
            stage_ms[stage[i]] += ms;
        }
    }
    return true;
}

}  // namespace

namespace {

constexpr int64_t kTuneMinQueries = 1024;   // smaller batches keep the default launch settings

// "arch/cus|metric|dim|pivots|fanout|log2(nq)|knn": the shape a tuned
// setting belongs to
std::string tune_key(const gts_index *idx, int64_t nq, bool knn)
{
    static std::mutex mu;
    static std::map<int, std::string> arch;
    int dev = 0;
    GTS_HIP(hipGetDevice(&dev));
    std::string a;
    {
        std::lock_guard<std::mutex> lk(mu);
        auto it = arch.find(dev);
        if (it == arch.end()) {
            hipDeviceProp_t p;
            GTS_HIP(hipGetDeviceProperties(&p, dev));
            std::string name = p.gcnArchName;
            name = name.substr(0, name.find(':'));
            it = arch.emplace(dev, name + "/" + std::to_string(p.multiProcessorCount)).first;
        }
        a = it->second;
    }
    int lg = 0;
    while (((int64_t)1 << (lg + 1)) <= nq) lg++;
    const IndexData &d = idx->data;
    return a + "|" + std::to_string(d.metric) + "|" + std::to_string(d.dim) + "|" + std::to_string(d.m) + "|" +
           std::to_string(d.tree.fanout) + "|" + std::to_string(lg) + "|" + (knn ? "1" : "0");
}

}  // namespace

void tune_cache_load(gts_index *idx)
{
    if (idx->tune_cache.empty()) return;
    FILE *f = std::fopen(idx->tune_cache.c_str(), "r");
    if (!f) return;
    char key[512];
    int w = 0, g = 0;
    std::lock_guard<std::mutex> lk(idx->tune_mu);
    while (std::fscanf(f, "%511s %d %d", key, &w, &g) == 3)
        if (w >= 0 && w < LaunchTuner::kWindows && g >= 0 && g < LaunchTuner::kGrids)
            idx->tuned[key] = TuneSetting{w, g};
    std::fclose(f);
}

// (caller holds tune_mu)  Entries of other shapes already in the file are
// kept; the file is replaced in one rename.
void tune_cache_store(gts_index *idx)
{
    if (idx->tune_cache.empty()) return;
    std::map<std::string, TuneSetting> all;
    if (FILE *f = std::fopen(idx->tune_cache.c_str(), "r")) {
        char key[512];
        int w = 0, g = 0;
        while (std::fscanf(f, "%511s %d %d", key, &w, &g) == 3)
            if (w >= 0 && w < LaunchTuner::kWindows && g >= 0 && g < LaunchTuner::kGrids) all[key] = TuneSetting{w, g};
        std::fclose(f);
    }
    for (const auto &e : idx->tuned) all[e.first] = e.second;
    const std::string tmp = idx->tune_cache + ".tmp";
    FILE *f = std::fopen(tmp.c_str(), "w");
    if (!f) return;   // an unwritable cache only loses the remembered settings
    for (const auto &e : all) std::fprintf(f, "%s %d %d\n", e.first.c_str(), e.second.window, e.second.grid);
    const bool ok = std::fclose(f) == 0;
    if (ok) std::rename(tmp.c_str(), idx->tune_cache.c_str());
}

size_t staging_bytes(int64_t nq) { return PinLayout(nq).bytes; }

void search(gts_index *idx, QueryCtx *cx, const gts_objects *Q, const float *radius, const int32_t *kin,
            const gts_query_opts *opts, gts_result *out, const NoAllocOut *na)
{
    const double t_start = now_ms();
    bool tune_trial = false;   // this call tries a tuner setting
    GTS_CHECK(out != nullptr, GTS_EINVAL, "null result");
    GTS_CHECK(Q != nullptr, GTS_EINVAL, "null queries");
    hipStream_t st = cx->stream;
    IndexData &d = idx->data;
    const bool l2 = d.metric == GTS_L2_F32;
    const int mpad = d.tree.mpad;
    Batch b;
    b.nq = Q->n;
    GTS_CHECK(b.nq >= 0, GTS_EINVAL, "negative query count");
    GTS_CHECK(b.nq < ((int64_t)1 << 31), GTS_ENOTSUP, "too many queries in one call");
    b.mode = opts ? opts->mode : GTS_MODE_BATCHED;
    GTS_CHECK(b.mode == GTS_MODE_BATCHED || b.mode == GTS_MODE_PLAIN, GTS_EINVAL, "bad mode");
    b.precision = opts && opts->precision != GTS_PRECISION_DEFAULT ? opts->precision : idx->opts.precision;
    if (b.precision == GTS_PRECISION_DEFAULT) b.precision = GTS_BF16_GUARDED;
    GTS_CHECK(b.precision == GTS_BF16_GUARDED || b.precision == GTS_FP32, GTS_EINVAL, "bad precision");
    GTS_CHECK(!opts || (opts->flags & ~(GTS_QF_CHECK_BOUND | GTS_QF_NO_PRUNE)) == 0, GTS_EINVAL,
              "unknown gts_query_opts.flags bits");
    b.check_bound = opts && (opts->flags & GTS_QF_CHECK_BOUND);
    b.no_prune = opts && (opts->flags & GTS_QF_NO_PRUNE);
    // tuned launch settings of the batched bf16 L2 path (answers never depend on them)
    std::string tkey;
    TuneSetting tset;
    // (batches under kTuneMinQueries take the defaults: their time is mostly
    // launch and host work, so trials there measure noise, and a server's
    // many small batch sizes would each pay for a full set of trials)
    const bool tunable = d.metric == GTS_L2_F32 && !idx->l1 && b.mode == GTS_MODE_BATCHED &&
                         b.precision == GTS_BF16_GUARDED && d.lpad > 0 && d.dim <= kMaxMfmaDim &&
                         b.nq >= kTuneMinQueries;
    if (tunable && cx->graph) {
        // a recorded graph takes the settings eager calls of its shape have
        // settled on (the kNN key: its queries may hold kNN), else the defaults
        const std::string gkey = tune_key(idx, b.nq, true);
        {
            std::lock_guard<std::mutex> lk(idx->tune_mu);
            auto it = idx->tuned.find(gkey);
            if (it != idx->tuned.end()) tset = it->second;
        }
        b.sweep_grid_per_cu = LaunchTuner::kGridPerCu[tset.grid];
    } else if (tunable) {
        bool knn = false;
        for (int64_t q = 0; q < b.nq && !knn; q++) knn = kin && kin[q] > 0;
        tkey = tune_key(idx, b.nq, knn);
        TuneSetting known;
        bool have = false;
        {
            std::lock_guard<std::mutex> lk(idx->tune_mu);
            auto it = idx->tuned.find(tkey);
            if (it != idx->tuned.end()) {
                known = it->second;
                have = true;
            }
        }
        tset = cx->tuner.pick(tkey, knn, have ? &known : nullptr, &tune_trial);
        b.sweep_grid_per_cu = LaunchTuner::kGridPerCu[tset.grid];
    }
    const int rloc = opts && (opts->result_location == GTS_HOST || opts->result_location == GTS_DEVICE)
                         ? opts->result_location
                         : Q->location;
    const int64_t nq = b.nq;
    // per-query kind, radius, k (a graph-mode search reads them on the device)
    const bool gmode = cx->graph;
    std::vector<int32_t> hk(gmode ? 0 : nq, 0);
    std::vector<float> hbase(gmode ? 0 : nq, 0.f);
    if (gmode) {
        GTS_CHECK(na != nullptr && cx->arena != nullptr && cx->gstatus != nullptr, GTS_EINVAL,
                  "graph-mode search without its fixed buffers");
        GTS_CHECK(d.metric == GTS_L2_F32, GTS_ENOTSUP, "search plans take vector indexes");
        GTS_CHECK(radius != nullptr && kin != nullptr, GTS_EINVAL, "graph-mode search needs radius and k arrays");
        b.any_knn = true;   // (unknown on the host: the kNN stages run, k = 0 queries skip them)
    }
    for (int64_t q = 0; q < (gmode ? 0 : nq); q++) {
        const int kk = kin ? kin[q] : 0;
        if (kin && kk < 0) fail(GTS_EINVAL, "k must be >= 1");
        if (kk > 0) {
            hk[q] = kk;
            b.any_knn = true;
        } else {
            GTS_CHECK(radius != nullptr, GTS_EINVAL, "radius array required for range queries");
            const float r = radius[q];
            GTS_CHECK(std::isfinite(r) && r >= 0.f, GTS_EINVAL, "radius must be finite and >= 0");
            // angular: the chord between unit vectors at angle r, 2 sin(r / 2)
            hbase[q] = idx->angular ? (float)(2.0 * std::sin(std::min((double)r, M_PI) / 2.0)) : r;
            b.max_radius = std::max(b.max_radius, r);
        }
    }
    if (na) {
        GTS_CHECK(cx->arena != nullptr, GTS_EINVAL, "no-allocation search without its arena");
        GTS_CHECK(gmode || nq <= kNoAllocMaxQueries, GTS_EINVAL,
                  "the no-allocation search takes at most " + std::to_string(kNoAllocMaxQueries) + " queries");
        GTS_CHECK(nq == 0 || Q->location == GTS_DEVICE, GTS_EINVAL, "the no-allocation search takes device queries");
        GTS_CHECK(b.mode == GTS_MODE_BATCHED, GTS_EINVAL, "the no-allocation search runs the batched form");
        GTS_CHECK(na->offsets != nullptr && (gmode || na->total != nullptr) && na->capacity >= 0, GTS_EINVAL,
                  "no-allocation output buffers");
        GTS_CHECK(na->capacity == 0 || (na->ids != nullptr && na->dist != nullptr), GTS_EINVAL,
                  "no-allocation output buffers");
        cx->timing = false;   // events would be created on first use
    }
    cx->stats = gts_stats{};
    cx->stats.nq = nq;
    std::memset(out, 0, sizeof(*out));
    out->nq = nq;
    out->metric = idx->angular ? GTS_COSINE_F32 : idx->l1 ? GTS_L1_F32 : d.metric;
    out->location = rloc;
    double stage_ms[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    if (cx->timing && !cx->ev[0])
        for (int i = 0; i < 9; i++) GTS_HIP(hipEventCreate(&cx->ev[i]));
    rec(cx, 0);
    const PinLayout pl(nq);
    uint8_t *pin = static_cast<uint8_t *>(cx->pinned(pl.bytes));
    GTS_CHECK(pin != nullptr, GTS_ENOMEM, "pinned host staging allocation failed");

    // ---- queries into the workspace -----------------------------------------------
    // query rows padded by one extra tile: a group that starts inside a tile
    // still reads whole tiles of fragments
    const int64_t ntiles_all = (nq + kQTile - 1) / kQTile;
    const int64_t nqpad = ntiles_all * kQTile + kQTile;
    b.ntiles_all = ntiles_all;
    wsp<float>(cx, W_QP, (size_t)nqpad * mpad);
    float *base = wsp<float>(cx, W_BASE, nqpad);
    wsp<float>(cx, W_T, nqpad);
    wsp<float>(cx, W_THR, nqpad);
    int32_t *kq = wsp<int32_t>(cx, W_KQ, nqpad);
    int32_t *home = wsp<int32_t>(cx, W_HOME, nqpad);
    unsigned long long *counters = wsp<unsigned long long>(cx, W_COUNTERS, k::kCounterWords);
    k::fill_u32(reinterpret_cast<uint32_t *>(counters), 2 * k::kCounterWords, 0u, st);
    if (nq > 0 && gmode) {
        k::query_params(radius, kin, nq, idx->angular, base, kq, cx->gstatus, st);
    } else if (nq > 0) {
        GTS_HIP(hipMemcpyAsync(base, hbase.data(), nq * sizeof(float), hipMemcpyHostToDevice, st));
        GTS_HIP(hipMemcpyAsync(kq, hk.data(), nq * sizeof(int32_t), hipMemcpyHostToDevice, st));
    }
    const hipMemcpyKind in_kind = Q->location == GTS_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    k::QueryL2 qv{};
    const int32_t *hqlen = nullptr;   // query string lengths (EDIT), caller order, pinned
    k::QueryEdit qe{};
    if (nq > 0 && l2) {
        GTS_CHECK(Q->dim == d.dim, GTS_EINVAL, "query dimension differs from the index");
        GTS_CHECK(Q->vecs != nullptr, GTS_EINVAL, "null query vectors");
        if (Q->location == GTS_HOST)
            for (int64_t i = 0; i < nq * d.dim; i++)
                GTS_CHECK(std::isfinite(Q->vecs[i]), GTS_EINVAL, "non-finite query value");
        float *Q32 = wsp<float>(cx, W_Q32, (size_t)nqpad * d.dp);
        k::fill_u32(reinterpret_cast<uint32_t *>(Q32), (int64_t)nqpad * d.dp, 0u, st);
        rows_to_device(Q32, d.dp, Q->vecs, d.dim, nq, Q->location == GTS_DEVICE, st);
        if (idx->angular || Q->location == GTS_DEVICE) {
            // device queries are checked on the device (a non-finite value
            // is flagged and replaced by zero, so that no later kernel sees
            // it); the flag is read with the first candidate counts
            uint32_t *bad = wsp<uint32_t>(cx, W_BADQ, 1);
            k::fill_u32(bad, 1, 0u, st);
            if (Q->location == GTS_DEVICE) k::check_finite(Q32, nq, d.dim, d.dp, bad, st);
            if (idx->angular) k::normalize_rows(Q32, nq, d.dim, d.dp, bad, st);
            b.check_q = true;
        }
        uint16_t *Q16 = wsp<uint16_t>(cx, W_Q16, (size_t)nqpad * d.ksteps * 32);
        float *qn = wsp<float>(cx, W_QN, nqpad);
        float *qerr = wsp<float>(cx, W_QE, nqpad);
        k::rows_bf16(Q32, nq, nqpad, d.dim, d.dp, d.ksteps, Q16, qn, qerr, 0.f, st);
        k::dist_l2_pivots(Q32, nq, d.P32.as<float>(), d.m, mpad, d.dp, cx->ws[W_QP].as<float>(), 1, mpad, st,
                          idx->l1);
        qv = k::QueryL2{Q32, Q16, qn, qerr};
    } else if (nq > 0) {
        GTS_CHECK(Q->offsets != nullptr, GTS_EINVAL, "null query offsets");
        int64_t *hoff = reinterpret_cast<int64_t *>(pin + pl.in_off);
        GTS_HIP(hipMemcpy(hoff, Q->offsets, (nq + 1) * sizeof(int64_t),
                          Q->location == GTS_DEVICE ? hipMemcpyDeviceToHost : hipMemcpyHostToHost));
        GTS_CHECK(hoff[0] == 0, GTS_EINVAL, "query offsets[0] must be 0");
        int32_t *qlen = reinterpret_cast<int32_t *>(pin + pl.in_len);
        hqlen = qlen;
        for (int64_t q = 0; q < nq; q++) {
            const int64_t len = hoff[q + 1] - hoff[q];
            GTS_CHECK(len >= 0 && len <= d.max_strlen, GTS_EINVAL, "query string length out of range");
            qlen[q] = (int32_t)len;
            b.max_qlen = std::max(b.max_qlen, (int)len);
        }
        uint8_t *qc = wsp<uint8_t>(cx, W_QCHARS, std::max<int64_t>(hoff[nq], 1));
        if (hoff[nq]) {
            GTS_CHECK(Q->chars != nullptr, GTS_EINVAL, "null query bytes");
            GTS_HIP(hipMemcpyAsync(qc, Q->chars, hoff[nq], in_kind, st));
        }
        int64_t *qo = wsp<int64_t>(cx, W_QOFF, nqpad + 1);
        GTS_HIP(hipMemcpyAsync(qo, hoff, (nq + 1) * sizeof(int64_t), hipMemcpyHostToDevice, st));
        int32_t *ql = wsp<int32_t>(cx, W_QLEN, nqpad);
        GTS_HIP(hipMemcpyAsync(ql, qlen, nq * sizeof(int32_t), hipMemcpyHostToDevice, st));
        uint64_t *peq = wsp<uint64_t>(cx, W_PEQ, (size_t)nqpad * idx->arows * 4);
        k::build_peq(qc, qo, nq, idx->lut.as<uint8_t>(), idx->arows, peq, st);
        k::dist_edit_pivots_f32(qc, qo, nq, d.pchars.as<uint8_t>(), d.poff.as<int32_t>(), d.m, mpad,
                                cx->ws[W_QP].as<float>(), 1, mpad, idx->lut.as<uint8_t>(), idx->arows, st);
        qe = k::QueryEdit{qc, qo, peq};
    }
    // ---- what the batch sees ------------------------------------------------------
    // Outside a server batch every query sees the index as it is now.  A
    // server batch spans updates: its queries carry admission epochs, the
    // producers run on the tombstones of the earliest epoch (a superset of
    // every query's live set, each candidate checked against its query's
    // epoch when grouped), the kNN bounds on those of the latest (a subset:
    // the k-th distance over it bounds every query's), and it scans the cache
    // slots filled at its admission.
    // (a server batch reads none of the update counters: the scheduler
    // changes them while the batch runs)
    b.tomb_prod = b.tomb_bound = d.tomb.as<uint32_t>();
    const SnapView &sv = cx->view;
    if (!sv.on) {
        b.e_now = idx->epoch;
        b.cache_count = idx->cache.n_live > 0 ? idx->cache.count : 0;
    } else if (nq > 0) {
        GTS_CHECK((int64_t)sv.qep.size() == nq && sv.e_min <= sv.e_max, GTS_EINVAL, "inconsistent admission epochs");
        uint32_t *qep = wsp<uint32_t>(cx, W_QEP, nqpad);
        GTS_HIP(hipMemcpyAsync(qep, sv.qep.data(), nq * sizeof(uint32_t), hipMemcpyHostToDevice, st));
        uint32_t *tmin = wsp<uint32_t>(cx, W_TMIN, d.tomb_words);
        k::tomb_bits(d.del_ep.as<uint32_t>(), d.n, sv.e_min, tmin, d.tomb_words, st);
        b.tomb_prod = b.tomb_bound = tmin;
        if (sv.e_max != sv.e_min) {
            uint32_t *tmax = wsp<uint32_t>(cx, W_TMAX, d.tomb_words);
            k::tomb_bits(d.del_ep.as<uint32_t>(), d.n, sv.e_max, tmax, d.tomb_words, st);
            b.tomb_bound = tmax;
        }
        b.qep = qep;
        b.cache_count = sv.cache_count;
    }

    // ---- home leaves and query order ----------------------------------------------
    // Queries are grouped into tiles by their home (nearest leaf pivot for L2,
    // nearest cluster centre in chain order for edit distance) so that a
    // tile's queries share surviving leaves; answers are returned in the
    // caller's order.
    k::TreeView tv{d.tree.box_aos.as<float>(), d.tree.box_lo.as<float>(), d.tree.box_hi.as<float>(),
                   d.tree.leaf_first.as<int32_t>(), d.tree.leaf_cnt.as<int32_t>(), d.tree.n_nodes,
                   d.tree.n_leaves, d.tree.leaf0, d.tree.fanout, d.tree.levels, mpad};
    k::EditView oe{d.chars.as<uint8_t>(), d.soff.as<int32_t>(), d.n, idx->lut.as<uint8_t>(), idx->arows};
    int32_t *near = nullptr;
    bool permuted = false;   // position i of the batch holds caller query perm[i] (W_PERM)
    // Edit distance (batched): the kNN bound, the thresholds and the cell test
    // run in the caller's order; a query's home is its first passing cell, and
    // the cell masks follow the queries into the grouped order.
    const bool edit_cells = !l2 && b.mode == GTS_MODE_BATCHED && d.n_centres > 0 && nq > 0;
    const float delta = (float)((d.dim + 8) * 5.9604645e-8);
    k::CellView cv{d.cchars.as<uint8_t>(), d.coff.as<int32_t>(), d.cellR.as<float>(), d.cell_box.as<float>(),
                   d.cell_len.as<int32_t>(), d.n_centres, d.cell_dist.as<uint8_t>(), d.qg_off.as<int32_t>(),
                   d.qg_cell.as<int32_t>()};
    int32_t *qcells0 = nullptr, *qcnt0 = nullptr;   // passing cells per position of the length order
    // the cell test runs on the queries in length order (a stable counting
    // sort), so that the tiles' patterns have similar word counts; dpos[q] =
    // position of query q in that order
    int32_t *dpos = nullptr;
    if (edit_cells) {
        int32_t *order = reinterpret_cast<int32_t *>(pin + pl.in_ord);
        int32_t *pos_of = reinterpret_cast<int32_t *>(pin + pl.in_pos);
        std::vector<int64_t> at(kMaxStrlen + 2, 0);
        for (int64_t q = 0; q < nq; q++) at[hqlen[q] + 1]++;
        for (int l = 0; l <= kMaxStrlen; l++) at[l + 1] += at[l];
        for (int64_t q = 0; q < nq; q++) {
            const int64_t p = at[hqlen[q]]++;
            order[p] = (int32_t)q;
            pos_of[q] = (int32_t)p;
        }
        int32_t *dorder = wsp<int32_t>(cx, W_ORDER, nq);
        GTS_HIP(hipMemcpyAsync(dorder, order, nq * sizeof(int32_t), hipMemcpyHostToDevice, st));
        dpos = wsp<int32_t>(cx, W_POSOF, nq);
        GTS_HIP(hipMemcpyAsync(dpos, pos_of, nq * sizeof(int32_t), hipMemcpyHostToDevice, st));
        int32_t *piv = wsp<int32_t>(cx, W_PIV, (size_t)2 * nq);
        k::edit_pivot(oe, qe, nq, cv, piv, piv + nq, st);
        if (b.any_knn)
            k::bound_edit(tv, oe, qe, cx->ws[W_QP].as<float>(), kq, nq, b.tomb_bound, 512, base, home, piv,
                          d.cell_leaf.as<int32_t>(), st);
        k::thresholds(base, cx->ws[W_QP].as<float>(), kq, nq, mpad, 1, delta, d.pt_max, cx->ws[W_T].as<float>(),
                      cx->ws[W_THR].as<float>(), wsp<float>(cx, W_CUT, nqpad), st);
        qcells0 = wsp<int32_t>(cx, W_QCELLS0, (size_t)nq * k::kQueryCells);
        qcnt0 = wsp<int32_t>(cx, W_QCNT0, nq);
        k::edit_cell_test(oe, qe, cx->ws[W_QLEN].as<int32_t>(), cx->ws[W_QP].as<float>(), mpad,
                          cx->ws[W_T].as<float>(), nq, b.max_qlen, cv, piv, piv + nq, qcells0, qcnt0, counters,
                          dorder, st);
    }
    // the nearest-leaf search and the leaf-window kNN bound run on bf16 MFMA
    // fragments of at most kMaxMfmaDim coordinates; wider rows use the tree
    // descent bound and keep the caller's order
    const bool leaf_mfma = l2 && d.lpad > 0 && d.dim <= kMaxMfmaDim && !idx->l1;
    if (nq > 1 && leaf_mfma) {
        // home = nearest leaf pivot; the order comes from a device sort
        near = wsp<int32_t>(cx, W_NEAR, (size_t)nqpad * k::kNearLeaves);
        k::leaf_near(d.PL16t.as<uint16_t>(), d.pln.as<float>(), d.lpad, d.ksteps, qv.Q16t, nq, near, st);
        const size_t tb = k::home_sort_bytes(nq, d.lpad);
        int32_t *dperm = wsp<int32_t>(cx, W_PERM, nq);
        k::home_sort(near, k::kNearLeaves, nq, d.lpad, reinterpret_cast<uint32_t *>(home),
                     wsp<uint32_t>(cx, W_HOME2, nq), dperm,
                     wsp<uint8_t>(cx, W_SORT_TMP, tb), tb, st);
        permuted = true;
    } else if (nq > 1 && edit_cells) {
        // home = first passing cell in chain order (per position of the length
        // order, then per query); the batch order is a stable device sort by it
        k::first_cell(qcells0, qcnt0, d.n_centres, nq, home, st);
        int32_t *homec = wsp<int32_t>(cx, W_HOMEC, nq);
        k::gather_i32(home, dpos, nq, 1, homec, st);
        const size_t tb = k::home_sort_bytes(nq, (int64_t)d.n_centres + 1);
        int32_t *dperm = wsp<int32_t>(cx, W_PERM, nq);
        k::home_sort(homec, 1, nq, (int64_t)d.n_centres + 1, reinterpret_cast<uint32_t *>(home),
                     wsp<uint32_t>(cx, W_HOME2, nq), dperm, wsp<uint8_t>(cx, W_SORT_TMP, tb), tb, st);
        permuted = true;
    }
    if (permuted) {
        // everything per query follows the permutation on the device: one
        // gather into partner buffers, which then trade places with the
        // originals (no copies back)
        const int32_t *dperm = cx->ws[W_PERM].as<int32_t>();
        float *pb = wsp<float>(cx, W_PBASE, nqpad);
        int32_t *pk = wsp<int32_t>(cx, W_PKQ, nqpad);
        float *pqp = wsp<float>(cx, W_PQP, (size_t)nqpad * mpad);
        float *pq32 = l2 ? wsp<float>(cx, W_PQ32, (size_t)nqpad * d.dp) : nullptr;
        int32_t *pnear = near ? wsp<int32_t>(cx, W_PNEAR, (size_t)nqpad * k::kNearLeaves) : nullptr;
        k::permute_queries(dperm, nq, base, pb, kq, pk, cx->ws[W_QP].as<float>(), pqp, mpad, l2 ? qv.Q32 : nullptr,
                           pq32, d.dp, near, pnear, k::kNearLeaves, st);
        if (b.qep) {
            uint32_t *pq = wsp<uint32_t>(cx, W_PQEP, nqpad);
            k::gather_i32(reinterpret_cast<const int32_t *>(b.qep), dperm, nq, 1, reinterpret_cast<int32_t *>(pq), st);
            std::swap(cx->ws[W_QEP], cx->ws[W_PQEP]);
            b.qep = cx->ws[W_QEP].as<uint32_t>();
        }
        std::swap(cx->ws[W_BASE], cx->ws[W_PBASE]);
        std::swap(cx->ws[W_KQ], cx->ws[W_PKQ]);
        std::swap(cx->ws[W_QP], cx->ws[W_PQP]);
        base = cx->ws[W_BASE].as<float>();
        kq = cx->ws[W_KQ].as<int32_t>();
        if (near) {
            std::swap(cx->ws[W_NEAR], cx->ws[W_PNEAR]);
            near = cx->ws[W_NEAR].as<int32_t>();
        }
        if (l2) {
            std::swap(cx->ws[W_Q32], cx->ws[W_PQ32]);
            qv.Q32 = cx->ws[W_Q32].as<float>();
            k::rows_bf16(qv.Q32, nq, nqpad, d.dim, d.dp, d.ksteps, const_cast<uint16_t *>(qv.Q16t),
                         const_cast<float *>(qv.qn), const_cast<float *>(qv.qe), 0.f, st);
        } else {
            // strings in the new order: lengths gathered, offsets scanned,
            // bytes gathered; then their match tables (all on the device)
            const int64_t total = reinterpret_cast<const int64_t *>(pin + pl.in_off)[nq];
            int32_t *nlen = wsp<int32_t>(cx, W_PLEN, nqpad);
            int64_t *noff = wsp<int64_t>(cx, W_POFF, nqpad + 1);
            uint8_t *nchars = wsp<uint8_t>(cx, W_PCHARS, std::max<int64_t>(total, 1));
            k::gather_i32(cx->ws[W_QLEN].as<int32_t>(), dperm, nq, 1, nlen, st);
            k::scan_u32(reinterpret_cast<const uint32_t *>(nlen), nq, noff, st);
            k::gather_strings(qe.chars, qe.off, dperm, nq, noff, nchars, st);
            k::build_peq(nchars, noff, nq, idx->lut.as<uint8_t>(), idx->arows, const_cast<uint64_t *>(qe.peq), st);
            std::swap(cx->ws[W_QLEN], cx->ws[W_PLEN]);
            std::swap(cx->ws[W_QOFF], cx->ws[W_POFF]);
            std::swap(cx->ws[W_QCHARS], cx->ws[W_PCHARS]);
            qe.chars = nchars;
            qe.off = noff;
        }
    }
    if (edit_cells) {
        // cell lists from length order to the batch order: batch position i
        // holds caller query perm[i], tested at position dpos[perm[i]]
        const int32_t *dcomp = dpos;
        if (permuted) {
            int32_t *c2 = wsp<int32_t>(cx, W_ORDER, nq);
            k::gather_i32(dpos, cx->ws[W_PERM].as<int32_t>(), nq, 1, c2, st);
            dcomp = c2;
        }
        k::gather_i32(qcells0, dcomp, nq, k::kQueryCells, wsp<int32_t>(cx, W_QCELLS, (size_t)nq * k::kQueryCells),
                      st);
        k::gather_i32(qcnt0, dcomp, nq, 1, wsp<int32_t>(cx, W_QCNT, nq), st);
    }
    rec(cx, 1);

    // ---- kNN bound ------------------------------------------------------------------
    if (nq > 0 && b.any_knn && !edit_cells) {
        if (leaf_mfma) {
            if (!near) {
                near = wsp<int32_t>(cx, W_NEAR, (size_t)nqpad * k::kNearLeaves);
                k::leaf_near(d.PL16t.as<uint16_t>(), d.pln.as<float>(), d.lpad, d.ksteps, qv.Q16t, nq, near, st);
            }
            const int window = LaunchTuner::kWindow[tset.window];
            cx->stats.bound_window = window;
            // bf16 MFMA bounds over block-shared windows; the exact window
            // kernel takes the queries those leave unbounded
            k::bound_mfma(d.X16t.as<uint16_t>(), d.xn.as<float>(), d.xe.as<float>(), d.n, d.ksteps, near,
                          d.tree.leaf_first.as<int32_t>(), d.tree.leaf_cnt.as<int32_t>(), qv.Q16t, qv.qn, qv.qe, kq,
                          nq, b.tomb_bound, window, base, counters, st);
            k::bound_near(near, d.tree.leaf_first.as<int32_t>(), d.tree.leaf_cnt.as<int32_t>(), d.X32.as<float>(),
                          d.dp, qv.Q32, kq, nq, b.tomb_bound, window, base, counters, st, true);
        } else if (l2) {
            k::L2View ov{d.X32.as<float>(), d.xn.as<float>(), d.xe.as<float>(), d.X16t.as<uint16_t>(), d.n, d.npad,
                         d.dim, d.dp, d.ksteps};
            k::bound_l2(tv, ov, qv, cx->ws[W_QP].as<float>(), kq, nq, b.tomb_bound, 256, base, home, st, idx->l1);
        } else {
            k::bound_edit(tv, oe, qe, cx->ws[W_QP].as<float>(), kq, nq, b.tomb_bound, 256, base, home, nullptr,
                          nullptr, st);
        }
    }
    if (nq > 0)
        k::thresholds(base, cx->ws[W_QP].as<float>(), kq, nq, mpad, l2 ? 0 : 1, delta, d.pt_max,
                      cx->ws[W_T].as<float>(), cx->ws[W_THR].as<float>(), wsp<float>(cx, W_CUT, nqpad), st);
    if (l2 && !idx->l1) k::sum_pad(cx->ws[W_T].as<float>(), qv.qe, nq, nqpad, wsp<float>(cx, W_TQE, nqpad), st);
    rec(cx, 2);
    if (cx->timing && nq > 0) {
        GTS_HIP(hipStreamSynchronize(st));
        float ms;
        GTS_HIP(hipEventElapsedTime(&ms, cx->ev[0], cx->ev[1]));
        stage_ms[GTS_STAGE_PREP] += ms;
        GTS_HIP(hipEventElapsedTime(&ms, cx->ev[1], cx->ev[2]));
        stage_ms[GTS_STAGE_BOUND] += ms;
    }

    // ---- groups of whole tiles under the budget -------------------------------------
    int64_t budget = opts && opts->mem_budget_bytes > 0 ? opts->mem_budget_bytes : idx->opts.mem_budget_bytes;
    if (budget <= 0) budget = (int64_t)1 << 32;
    const int64_t per_cand = 2 * (int64_t)sizeof(k::Cand) + (int64_t)sizeof(uint64_t);
    int64_t cap = std::max<int64_t>(budget / per_cand, 1024);
    if (cx->arena && nq > 0) {
        // what the group needs besides its per-candidate buffers (candidates,
        // grouped copy, sorted keys, long-segment sort space: 56 bytes each)
        const int64_t ntl = (nq + kQTile - 1) / kQTile;
        const Tree &tr = d.tree;
        size_t reserve = (size_t)1 << 20;
        auto add = [&](size_t bytes) { reserve += Arena::align(std::max<size_t>(bytes, 64)); };
        add(kSmallWords * sizeof(uint32_t));
        add((size_t)tr.n_leaves * ntl * sizeof(uint64_t));           // leaf masks
        add((size_t)tr.n_leaves * ntl * 2 * sizeof(int32_t));       // (leaf, tile) items
        add((size_t)d.n_slabs * ntl * sizeof(int32_t));              // sweep pairs
        add((size_t)d.n_slabs * ntl * sizeof(uint64_t));
        add((size_t)d.n_slabs * ((ntl + k::kSweepItemTiles - 1) / k::kSweepItemTiles) * sizeof(int4));
        for (int i = 0; i < 4; i++) add((size_t)(nq + 1) * sizeof(uint32_t));
        for (int i = 0; i < 3; i++) add((size_t)(nq + 1) * sizeof(int64_t));
        add((size_t)nq * sizeof(int32_t));
        // the device-side verification plan (need, class counts, order; need
        // offsets, scratch offsets)
        for (int i = 0; i < 3; i++) add((size_t)(nq + 1) * sizeof(uint32_t));
        for (int i = 0; i < 3; i++) add((size_t)(nq + 1) * sizeof(int64_t));
        add((size_t)k::kVerifyCursorWords * sizeof(uint32_t));   // the verification's work-queue cursors
        const size_t left = cx->arena->left();
        GTS_CHECK(left >= reserve + (size_t)56 * 1024, GTS_ENOMEM,
                  "the no-allocation scratch cannot hold this batch's work lists; use a smaller batch");
        cap = std::min<int64_t>(cap, (int64_t)((left - reserve) / 56));
    }
    std::vector<GroupOut> groups;
    std::vector<std::pair<int64_t, int64_t>> todo;  // (q0, ng), processed front to back
    if (nq > 0) todo.push_back({0, nq});
    if (permuted && !gmode)   // the order was made on the device: its copy lands by the next sync
        GTS_HIP(hipMemcpyAsync(pin + pl.perm, cx->ws[W_PERM].p, nq * sizeof(int32_t), hipMemcpyDeviceToHost, st));
    while (!todo.empty()) {
        auto [q0, ng] = todo.front();
        todo.erase(todo.begin());
        GroupOut go;
        // the whole batch in one group leaves its sorted keys in the workspace
        const bool direct = q0 == 0 && ng == nq;
        if (run_group(idx, cx, b, q0, ng, cap, direct, rloc == GTS_DEVICE, pin, pl, &go, stage_ms)) {
            groups.push_back(std::move(go));
            continue;
        }
        GTS_CHECK(!cx->arena, GTS_ENOMEM,
                  "the batch's candidates exceed the no-allocation scratch; use a smaller batch");
        const int64_t blocks = (ng + kQTile - 1) / kQTile;
        GTS_CHECK(blocks > 1, GTS_ENOMEM,
                  "the memory budget cannot hold the candidates of 64 queries; raise mem_budget_bytes");
        cx->stats.group_retries++;
        std::vector<std::pair<int64_t, int64_t>> parts;
        unsigned long long work = 0;
        for (unsigned long long w : go.tile_work) work += w;
        if ((int64_t)go.tile_work.size() == blocks && work > 0) {
            // consecutive tiles whose estimated candidates (the attempt's
            // count shared in proportion to each tile's pairs in surviving
            // leaves) fill three quarters of the budget
            const long double per = (long double)go.attempts / (long double)work;
            const long double target = 0.75L * (long double)cap;
            int64_t t0 = 0;
            long double acc = 0.0L;
            for (int64_t tt = 0; tt < blocks; tt++) {
                const long double c = per * (long double)go.tile_work[tt];
                if (tt > t0 && acc + c > target) {
                    parts.push_back({t0, tt});
                    t0 = tt;
                    acc = 0.0L;
                }
                acc += c;
            }
            parts.push_back({t0, blocks});
        }
        if (parts.size() < 2) parts = {{0, blocks / 2}, {blocks / 2, blocks}};   // halves
        for (size_t i = parts.size(); i-- > 0;) {
            const int64_t a = q0 + parts[i].first * kQTile;
            const int64_t e = std::min(q0 + ng, q0 + parts[i].second * kQTile);
            todo.insert(todo.begin(), {a, e - a});
        }
    }

    // ---- final CSR (caller's query order) ------------------------------------------------
    unsigned long long *hc = reinterpret_cast<unsigned long long *>(pin + pl.counters);
    if (na) {
        // no-allocation search: caller-order counts, their scan straight into
        // the caller's offsets, a capacity check, then the keys in place
        int64_t *htot = reinterpret_cast<int64_t *>(pin + pl.offs);
        if (gmode) {
            // a recorded graph: counts, their scan into the caller's offsets
            // (offsets[nq] = the answers), the keys written below the
            // capacity, then the status word; nothing read on the host
            uint32_t *cc = wsp<uint32_t>(cx, W_TMP2, nq);
            const int32_t *dperm = permuted ? cx->ws[W_PERM].as<int32_t>() : nullptr;
            k::perm_counts(cx->ws[W_OUTCNT].as<uint32_t>(), dperm, nq, cc, st);
            k::scan_u32(cc, nq, na->offsets, st);
            k::emit_result(cx->ws[W_OUTKEYS].as<uint64_t>(), cx->ws[W_QOFF64].as<int64_t>(),
                           cx->ws[W_OUTCNT].as<uint32_t>(), dperm, na->offsets, nq, 0, na->ids,
                           static_cast<float *>(na->dist), nullptr, st, na->capacity);
            k::plan_status(cx->gstatus, cx->ws[W_BADQ].as<uint32_t>(), nullptr, 0, na->offsets + nq, na->capacity, st);
            out->total = -1;
            return;
        }
        if (groups.empty()) {
            k::fill_u32(reinterpret_cast<uint32_t *>(na->offsets), 2 * (nq + 1), 0u, st);
        } else {
            uint32_t *cc = wsp<uint32_t>(cx, W_TMP2, nq);
            const int32_t *dperm = permuted ? cx->ws[W_PERM].as<int32_t>() : nullptr;
            k::perm_counts(cx->ws[W_OUTCNT].as<uint32_t>(), dperm, nq, cc, st);
            k::scan_u32(cc, nq, na->offsets, st);
        }
        GTS_HIP(hipMemcpyAsync(htot, na->offsets + nq, sizeof(int64_t), hipMemcpyDeviceToHost, st));
        GTS_HIP(hipMemcpyAsync(hc, counters, k::kCounterWords * sizeof(unsigned long long), hipMemcpyDeviceToHost, st));
        GTS_HIP(hipStreamSynchronize(st));
        const int64_t total = *htot;
        *na->total = total;
        GTS_CHECK(total <= na->capacity, GTS_ENOMEM,
                  "the answers (" + std::to_string(total) + ") exceed the output capacity (" +
                      std::to_string(na->capacity) + ")");
        if (total > 0) {
            const int32_t *dperm = permuted ? cx->ws[W_PERM].as<int32_t>() : nullptr;
            k::emit_result(cx->ws[W_OUTKEYS].as<uint64_t>(), cx->ws[W_QOFF64].as<int64_t>(),
                           cx->ws[W_OUTCNT].as<uint32_t>(), dperm, na->offsets, nq, l2 ? 0 : 1, na->ids,
                           static_cast<float *>(na->dist), static_cast<int32_t *>(na->dist), st);
            GTS_HIP(hipStreamSynchronize(st));
        }
        out->total = total;
    } else if (groups.size() == 1 && groups[0].total < 0) {
        // one group, result on the device, storage made while verify ran:
        // caller-order counts, their scan (the result's offsets) and the keys
        // written in place, then one synchronisation for the total
        ResultMem rm = std::move(groups[0].pre);
        auto *priv = new ResultPriv();
        priv->device = true;
        priv->offsets = rm.p;
        priv->ids = static_cast<uint8_t *>(rm.p) + rm.id_at;
        priv->dist = static_cast<uint8_t *>(rm.p) + rm.dist_at;
        rm.release();
        out->priv = priv;
        int64_t *doffs = static_cast<int64_t *>(priv->offsets);
        uint32_t *cc = reinterpret_cast<uint32_t *>(wsp<int32_t>(cx, W_TMP2, nq));
        const int32_t *dperm = permuted ? cx->ws[W_PERM].as<int32_t>() : nullptr;
        k::perm_counts(cx->ws[W_OUTCNT].as<uint32_t>(), dperm, nq, cc, st);
        k::scan_u32(cc, nq, doffs, st);
        k::emit_result(cx->ws[W_OUTKEYS].as<uint64_t>(), cx->ws[W_QOFF64].as<int64_t>(),
                       cx->ws[W_OUTCNT].as<uint32_t>(), dperm, doffs, nq, l2 ? 0 : 1,
                       static_cast<int64_t *>(priv->ids), static_cast<float *>(priv->dist),
                       static_cast<int32_t *>(priv->dist), st);
        int64_t *htot = reinterpret_cast<int64_t *>(pin + pl.offs);
        GTS_HIP(hipMemcpyAsync(htot, doffs + nq, sizeof(int64_t), hipMemcpyDeviceToHost, st));
        GTS_HIP(hipMemcpyAsync(hc, counters, k::kCounterWords * sizeof(unsigned long long), hipMemcpyDeviceToHost, st));
        GTS_HIP(hipStreamSynchronize(st));
        out->total = *htot;
        out->offsets = doffs;
        out->ids = static_cast<int64_t *>(priv->ids);
        if (l2) out->dist_f32 = static_cast<float *>(priv->dist);
        else out->dist_i32 = static_cast<int32_t *>(priv->dist);
    } else {
    // position i of the batch holds caller query pm[i]
    const int32_t *pm = !permuted ? nullptr : reinterpret_cast<const int32_t *>(pin + pl.perm);
    int64_t total = 0;
    for (auto &g : groups) total += g.total;
    int64_t *offs = reinterpret_cast<int64_t *>(pin + pl.offs);   // caller order, built in place
    {
        offs[0] = 0;
        int64_t i = 0;
        for (auto &g : groups)
            for (uint32_t c : g.counts) {
                offs[(pm ? pm[i] : i) + 1] = c;
                i++;
            }
        for (int64_t q = 0; q < nq; q++) offs[q + 1] += offs[q];
    }
    // one allocation holds offsets, ids and distances (made while verify ran
    // when the batch was one group)
    const size_t off_bytes = (nq + 1) * sizeof(int64_t);
    ResultMem rm;
    if (groups.size() == 1 && groups[0].pre.p && groups[0].pre.cap >= total) rm = std::move(groups[0].pre);
    else rm = result_alloc(nq, total, rloc == GTS_DEVICE);
    GTS_CHECK(rm.p != nullptr, GTS_ENOMEM, "result allocation failed");
    auto *priv = new ResultPriv();
    priv->device = rm.device;
    priv->offsets = rm.p;
    priv->ids = static_cast<uint8_t *>(rm.p) + rm.id_at;
    priv->dist = static_cast<uint8_t *>(rm.p) + rm.dist_at;
    rm.release();
    const int is_edit = l2 ? 0 : 1;
    // device copy of the caller-order offsets (the result's own array when it
    // lives on the device)
    int64_t *doffs = priv->device ? static_cast<int64_t *>(priv->offsets) : wsp<int64_t>(cx, W_OFF_ORIG, nq + 1);
    GTS_HIP(hipMemcpyAsync(doffs, offs, off_bytes, hipMemcpyHostToDevice, st));
    if (!priv->device) std::memcpy(priv->offsets, offs, off_bytes);
    int64_t *ids_d = priv->device ? static_cast<int64_t *>(priv->ids)
                                  : wsp<int64_t>(cx, W_RES_IDS, std::max<int64_t>(total, 1));
    uint32_t *dist_d = priv->device ? static_cast<uint32_t *>(priv->dist)
                                    : wsp<uint32_t>(cx, W_RES_DIST, std::max<int64_t>(total, 1));
    const int32_t *dperm = permuted ? cx->ws[W_PERM].as<int32_t>() : nullptr;
    if (groups.size() == 1 && groups[0].direct) {
        k::emit_result(cx->ws[W_OUTKEYS].as<uint64_t>(), cx->ws[W_QOFF64].as<int64_t>(),
                       cx->ws[W_OUTCNT].as<uint32_t>(), dperm, doffs, nq, is_edit, ids_d,
                       reinterpret_cast<float *>(dist_d), reinterpret_cast<int32_t *>(dist_d), st);
    } else {
        // group pieces in batch order, then un-permuted into place
        std::vector<int64_t> offs_b(nq + 1, 0);
        {
            int64_t q = 0;
            for (auto &g : groups)
                for (uint32_t c : g.counts) {
                    offs_b[q + 1] = offs_b[q] + c;
                    q++;
                }
        }
        int64_t *ids_b = wsp<int64_t>(cx, W_RES_IDS2, std::max<int64_t>(total, 1));
        uint32_t *dist_b = wsp<uint32_t>(cx, W_RES_DIST2, std::max<int64_t>(total, 1));
        int64_t at = 0;
        for (auto &g : groups) {
            if (g.total) {
                GTS_HIP(hipMemcpyAsync(ids_b + at, g.ids.p, g.total * sizeof(int64_t), hipMemcpyDeviceToDevice, st));
                GTS_HIP(hipMemcpyAsync(dist_b + at, g.dist.p, g.total * sizeof(float), hipMemcpyDeviceToDevice, st));
            }
            at += g.total;
        }
        if (total > 0) {
            if (permuted) {
                int64_t *dob = wsp<int64_t>(cx, W_RESOFF, nq + 1);
                GTS_HIP(hipMemcpyAsync(dob, offs_b.data(), off_bytes, hipMemcpyHostToDevice, st));
                k::unpermute(dob, doffs, dperm, nq, ids_b, dist_b, ids_d, dist_d, st);
            } else {
                GTS_HIP(hipMemcpyAsync(ids_d, ids_b, total * sizeof(int64_t), hipMemcpyDeviceToDevice, st));
                GTS_HIP(hipMemcpyAsync(dist_d, dist_b, total * sizeof(float), hipMemcpyDeviceToDevice, st));
            }
        }
    }
    if (!priv->device && total > 0) {
        GTS_HIP(hipMemcpyAsync(priv->ids, ids_d, total * sizeof(int64_t), hipMemcpyDeviceToHost, st));
        GTS_HIP(hipMemcpyAsync(priv->dist, dist_d, total * sizeof(float), hipMemcpyDeviceToHost, st));
    }
    GTS_HIP(hipMemcpyAsync(hc, counters, k::kCounterWords * sizeof(unsigned long long), hipMemcpyDeviceToHost, st));
    GTS_HIP(hipStreamSynchronize(st));
    out->total = total;
    out->offsets = static_cast<int64_t *>(priv->offsets);
    out->ids = static_cast<int64_t *>(priv->ids);
    if (l2) out->dist_f32 = static_cast<float *>(priv->dist);
    else out->dist_i32 = static_cast<int32_t *>(priv->dist);
    out->priv = priv;
    }

    // ---- counters ----------------------------------------------------------------------
    for (int c = 0; c < k::kCounters; c++) {   // sum the stripes into hc[c]
        unsigned long long v = 0;
        for (int j = 0; j < k::kStripes; j++) v += hc[((size_t)c * k::kStripes + j) * k::kStripeStride];
        hc[c] = v;   // slots 1..7 lie in the padding of counter 0's first stripe
    }
    cx->stats.node_tests = (int64_t)hc[0];
    if (cx->stats.leaf_pairs == 0) cx->stats.leaf_pairs = (int64_t)hc[1];
    cx->stats.tile_pairs = (int64_t)hc[2];
    cx->stats.verified = (int64_t)hc[3];
    cx->stats.bound_evals = (int64_t)hc[4];
    cx->stats.bound_violations = (int64_t)hc[k::CNT_BOUND_VIOL];
    cx->stats.own_pairs = (int64_t)hc[k::CNT_OWN_PAIRS];
    cx->stats.filter_objects = (int64_t)hc[k::CNT_FILTER_OBJS];
    cx->stats.results = out->total;
    for (int i = 0; i < 8; i++) cx->stats.ms_stage[i] = stage_ms[i];
    cx->stats.groups = (int64_t)groups.size();
    cx->stats.ms_total = now_ms() - t_start;
    TuneSetting settled;
    if (tune_trial && cx->tuner.record(tkey, cx->stats.ms_total / (double)nq, &settled)) {
        std::lock_guard<std::mutex> lk(idx->tune_mu);
        idx->tuned[tkey] = settled;
        tune_cache_store(idx);
    }
    cx->stats.tuning = cx->tuner.tuning() ? 1 : 0;
    cx->stats.sweep_grid_per_cu = b.sweep_grid_per_cu;
}

void free_result(gts_result *r)
{
    if (!r || !r->priv) return;
    auto *p = static_cast<ResultPriv *>(r->priv);
    // one allocation starting at the offsets holds the whole result
    if (p->offsets) (void)(p->device ? hipFree(p->offsets) : hipHostFree(p->offsets));
    delete p;
    std::memset(r, 0, sizeof(*r));
}

bool result_on_device(const gts_result *r)
{
    return r && r->priv && static_cast<const ResultPriv *>(r->priv)->device;
}

}  // namespace gts
