// Internal declarations shared by the host code and the kernel launchers of
// libgts.so.  Nothing here is part of the C ABI (see include/gts.h).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstring>
#include <memory>
#include <stdexcept>
#include <string>
#include <functional>
#include <map>
#include <mutex>
#include <vector>

#include "../../include/gts.h"

namespace gts {

// ---------------------------------------------------------------------------
// Errors: every internal failure throws gts::Error, which the C ABI layer
// turns into a status and a thread-local message.
// ---------------------------------------------------------------------------
struct Error : std::runtime_error {
    gts_status status;
    Error(gts_status s, const std::string &m) : std::runtime_error(m), status(s) {}
};

[[noreturn]] void fail(gts_status s, const std::string &msg);

#define GTS_HIP(call)                                                                   \
    do {                                                                                \
        hipError_t e_ = (call);                                                         \
        if (e_ != hipSuccess)                                                           \
            ::gts::fail(GTS_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

#define GTS_CHECK(cond, status, msg)                  \
    do {                                              \
        if (!(cond)) ::gts::fail((status), (msg));    \
    } while (0)

// ---------------------------------------------------------------------------
// Fixed shape parameters of the kernels.
// ---------------------------------------------------------------------------
constexpr int kWave = 64;           // CDNA wavefront
constexpr int kQTile = 64;          // queries per tile (one per lane of a wave)
constexpr int kSlab = 256;          // objects per MFMA slab (4 waves x 64 rows)
constexpr int kMaxPivots = 32;      // pivot table rows (padded to 8/16/32)
constexpr int kMaxMfmaDim = 128;    // largest L2 dimension on the MFMA path
constexpr int kMaxStrlen = 255;     // longest string (pivot table is uint8)
constexpr int kSortCap = 2048;      // edit distance: per-query keys sorted in LDS (more: global scratch)
constexpr int kSortCapL2 = 4096;    // L2: per-query keys sorted in LDS (more: global scratch)
constexpr int kWaveSortCap = 1024;  // L2: per-query keys one wave's LDS run holds
constexpr int kWorkspaceSlots = 80;   // named query buffers of an index
constexpr int kMaxCentres = 2048;      // farthest-first centres that order the leaves

// Device buffer owned by the index (hipMalloc / hipFree), or a view of
// memory owned elsewhere (owned = false: never freed here).
struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
    bool owned = true;
    DevBuf() = default;
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    DevBuf(DevBuf &&o) noexcept : p(o.p), bytes(o.bytes), owned(o.owned) { o.p = nullptr; o.bytes = 0; }
    DevBuf &operator=(DevBuf &&o) noexcept {
        if (this != &o) { release(); p = o.p; bytes = o.bytes; owned = o.owned; o.p = nullptr; o.bytes = 0; }
        return *this;
    }
    ~DevBuf() { release(); }
    void release() {
        if (p && owned) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
        owned = true;
    }
    void alloc(size_t b) {
        if (b <= bytes && p) return;
        release();
        if (b == 0) b = 16;
        hipError_t e = hipMalloc(&p, b);
        if (e != hipSuccess) {
            p = nullptr;
            fail(GTS_ENOMEM, "hipMalloc(" + std::to_string(b) + " bytes): " + hipGetErrorString(e));
        }
        bytes = b;
    }
    template <class T> T *as() const { return static_cast<T *>(p); }
};

// ---------------------------------------------------------------------------
// The index as it lives in HBM.  Objects are stored in leaf order: leaf j
// covers positions [leaf_first[j], leaf_first[j] + leaf_cnt[j]).
// ---------------------------------------------------------------------------
struct Tree {
    int32_t fanout = 2;
    int32_t levels = 0;          // partition layers; leaves are at this depth
    int64_t n_nodes = 1;         // (F^(levels+1) - 1) / (F - 1)
    int64_t n_leaves = 1;        // F^levels
    int64_t leaf0 = 0;           // node id of the first leaf
    int32_t mpad = 8;            // pivot rows padded to 8, 16 or 32
    DevBuf box_aos;              // float [n_nodes][2*mpad]: lo[0..mpad), hi[0..mpad)
    DevBuf box_lo, box_hi;       // float [mpad][n_nodes] (node-major lanes)
    DevBuf leaf_first, leaf_cnt; // int32 [n_leaves]
};

struct IndexData {
    int32_t metric = GTS_L2_F32;
    int64_t n = 0;               // objects in the tree (positions)
    int32_t m = 0;               // pivots
    // L2
    int32_t dim = 0;             // D
    int32_t dp = 0;              // float row stride of X32 (multiple of 4)
    int32_t ksteps = 0;          // bf16 K-steps of 32 (D padded to 32*ksteps)
    int64_t npad = 0;            // rows padded to a multiple of kSlab
    DevBuf X32;                  // float [npad][dp]
    DevBuf X16t;                 // bf16 MFMA A fragments [npad/16][ksteps][64][8]
    DevBuf xn;                   // float [npad] ||x16||^2 (padding rows: +inf)
    DevBuf xe;                   // float [npad] ||x16 - x32||
    DevBuf P32;                  // float [m][dp] pivot vectors
    DevBuf PT;                   // float [mpad][n] pivot distances (L2)
    int64_t lpad = 0;            // leaves padded to a multiple of 64
    DevBuf PL32;                 // float [lpad][dp] leaf pivot vectors
    DevBuf PL16t;                // bf16 fragments of the leaf pivots
    DevBuf pln, ple;             // float [lpad] ||p16||^2 (+inf: empty) and ||p16 - p||
    DevBuf leafR;                // float [lpad] max distance from the leaf pivot
    int64_t n_slabs = 0;
    DevBuf slab_emax, slab_nmax; // float [n_slabs]
    DevBuf slab_leaf_lo, slab_leaf_hi; // int32 [n_slabs]: leaves overlapping
    // EDIT
    int32_t max_strlen = kMaxStrlen;
    DevBuf chars;                // uint8 [total] strings in leaf order
    DevBuf soff;                 // int32 [n + 1]
    DevBuf PTe;                  // uint8 [mpad][n] pivot distances (SoA)
    DevBuf PTa;                  // uint8 [n][mpad] pivot distances (AoS)
    DevBuf pchars;               // uint8 pivot strings
    DevBuf poff;                 // int32 [m + 1]
    std::vector<std::string> pivot_str;
    DevBuf cchars;               // uint8 centre strings, in chain order
    DevBuf coff;                 // int32 [n_centres + 1]
    int32_t n_centres = 0;
    DevBuf cellR;                // float [n_centres] covering radius of each cell
    DevBuf cell_box;             // float [n_centres][2 * mpad] global pivot box
    DevBuf cell_len;             // int32 [n_centres][2] string length range
    DevBuf leaf_cell;            // int32 [n_leaves][2] first and last cell of a leaf
    DevBuf cell_leaf;            // int32 [n_centres][2] first and last leaf of a cell
    DevBuf cell_dist;            // uint8 [n_centres][n_centres] centre-to-centre distances
    DevBuf qg_off;               // int32 [kQgramBuckets + 1] centres per q-gram bucket (CSR)
    DevBuf qg_cell;              // int32 centres (chain rank) listed by bucket
    // both
    float pt_max = 0.f;          // largest pivot-table value
    DevBuf ids;                  // uint32 [n] id at each position
    DevBuf tomb;                 // uint32 [tomb_words] deleted positions (bit per position)
    DevBuf del_ep;               // uint32 [32 tomb_words] epoch of the update that deleted the
                                 // position (0xffffffff: live)
    int64_t tomb_words = 0;
    Tree tree;
};

// Streamed inserts not yet in the tree (the paper's cache list).
struct CacheList {
    int64_t cap = 0, count = 0;   // slots used (live or deleted)
    DevBuf X32;                   // float [cap][dp] (L2)
    DevBuf chars;                 // uint8 [cap * kMaxStrlen] (EDIT, fixed slots)
    DevBuf slen;                  // int32 [cap]
    DevBuf ids;                   // uint32 [cap]
    DevBuf ins_ep, del_ep;        // uint32 [cap] epochs of the slot's insert and delete
                                  // (del_ep 0xffffffff: live)
    DevBuf cp;                    // float [cap][mpad] distances to the global pivots (edit)
    std::vector<uint32_t> h_ids;
    std::vector<uint8_t> h_live;
    int64_t n_live = 0;           // live cached objects
};

// Host-side copy of everything needed to rebuild (the objects by id).
struct HostObjects {
    int32_t metric = GTS_L2_F32;
    int32_t dim = 0;
    std::vector<float> vecs;          // [count][dim]
    std::vector<uint8_t> chars;
    std::vector<int64_t> offsets{0};
    std::vector<uint32_t> ids;        // id of each stored object
    int64_t count() const { return (int64_t)ids.size(); }
    void clear() { vecs.clear(); chars.clear(); offsets.assign(1, 0); ids.clear(); }
    void append_from(const HostObjects &o, int64_t i) {
        if (metric == GTS_L2_F32) {
            vecs.insert(vecs.end(), o.vecs.begin() + i * dim, o.vecs.begin() + (i + 1) * dim);
        } else {
            chars.insert(chars.end(), o.chars.begin() + o.offsets[i], o.chars.begin() + o.offsets[i + 1]);
            offsets.push_back((int64_t)chars.size());
        }
        ids.push_back(o.ids[i]);
    }
};

// Build the tree and all device tables of `idx` over `objs` (ids given);
// objs becomes the index's host mirror (moved from).  A vector index may take
// its rows from `rows` (n rows of dp floats on the device, moved from) instead
// of objs.vecs.
void build_tree(gts_index *idx, HostObjects &objs, DevBuf *rows = nullptr);
// Rebuild over every live object (tree and cache), keeping ids; for a vector
// index, n_extra more rows already on the device (extra_rows, dp floats each)
// with their ids join.
void rebuild(gts_index *idx, DevBuf *extra_rows = nullptr, int64_t n_extra = 0, const uint32_t *extra_ids = nullptr);
// Copy n rows of dim floats (src, packed) into device rows of dp floats
// (dp >= dim; the dp - dim padding columns become zero).  Host sources are
// copied as one contiguous transfer (packed to the padded width on the host
// first when dp > dim) and have completed on return; device sources are
// copied in stream order.
void rows_to_device(float *dst, int dp, const float *src, int dim, int64_t n, bool src_on_device, hipStream_t st);
// Add the bytes of `chars` to the index alphabet (uploads the table when it
// changes; blocking).
void alphabet_add(gts_index *idx, const std::vector<uint8_t> &chars);
// Streamed updates.
void insert_objects(gts_index *idx, const HostObjects &objs, int64_t *out_ids);
// upload = false: host bookkeeping only (a rebuild follows).  A delete that
// leaves more than half of the tree's positions deleted rebuilds the index.
int64_t delete_ids(gts_index *idx, const int64_t *ids, int64_t n, bool upload = true);
// More than half of the tree deleted once `more` further positions are.
bool tree_mostly_deleted(const gts_index *idx, int64_t more = 0);
// Batch update: deletions, insertions (fresh ids into out_ids), one rebuild.
void update_batch(gts_index *idx, const HostObjects &ins, const int64_t *del, int64_t n_del, int64_t *out_ids,
                  int64_t *n_deleted);
// Per-stream query state: the workspace, timing events and statistics of
// the searches issued on one stream.  An index has a default context on its
// own stream; more contexts let searches of one index run concurrently (the
// index data is only read by a search).
// Online tuning of two launch settings of the batched L2 path, which trade
// work between stages and never change answers:
//   - the kNN bound window (objects per query whose exact distances bound
//     the k-th distance): small is cheap but leaves a loose bound and more
//     candidates downstream, large the reverse;
//   - the MFMA sweep's persistent grid (workgroups per CU): more overlaps
//     memory latency, fewer keeps the work-stealing tail short.
// A context tries each window (kNN batches only) on a few batches with the
// default grid, then each grid with the best window, and keeps the setting
// with the lowest time per query; each shape key keeps its own trials.  Settings are remembered per shape key
// (device, metric, dimension, pivots, fanout, log2 of the batch size, kNN
// present) in the index's table, which a tune-cache file can preload and
// which is written back when a key finishes tuning.
struct TuneSetting {
    int window = 1;                            // index into LaunchTuner::kWindow
    int grid = 1;                              // index into LaunchTuner::kGridPerCu
};
struct LaunchTuner {
    static constexpr int kWindows = 4;
    static constexpr int kGrids = 3;
    static constexpr int kTrials = 3;          // batches per setting (the fastest counts)
    static constexpr int kWindow[kWindows] = {128, 256, 512, 1024};
    static constexpr int kGridPerCu[kGrids] = {1, 2, 4};
    // trials of one shape key; a context tunes several keys at once, so
    // batches of changing size (a server's) do not restart each other's trials
    struct Progress {
        bool knn = false;
        int trial = 0;                         // trials done
        double ms_per_q[kWindows + kGrids] = {};
        TuneSetting best;
        int total() const { return (knn ? kWindows * kTrials : 0) + kGrids * kTrials; }
    };
    std::map<std::string, Progress> keys;      // keys still tuning
    bool last_tuning = false;                  // the last call's key was still tuning
    bool tuning() const { return last_tuning; }
    // The setting of a call on shape `k`; *trying is set when it is a trial.
    TuneSetting pick(const std::string &k, bool has_knn, const TuneSetting *known, bool *trying)
    {
        *trying = false;
        last_tuning = false;
        if (known) {
            keys.erase(k);
            return *known;
        }
        auto it = keys.find(k);
        if (it == keys.end()) {
            it = keys.emplace(k, Progress{}).first;
            it->second.knn = has_knn;
        }
        Progress &p = it->second;
        *trying = true;
        last_tuning = true;
        TuneSetting s = p.best;
        const int wt = p.knn ? kWindows * kTrials : 0;
        if (p.trial < wt) {
            s.window = p.trial % kWindows;
            s.grid = 1;
        } else {
            s.grid = (p.trial - wt) % kGrids;
        }
        return s;
    }
    // Time of a trial call on key `k`; returns true (and the setting in
    // *done) when `k` has just finished.
    bool record(const std::string &k, double ms_per_query, TuneSetting *done)
    {
        auto it = keys.find(k);
        if (it == keys.end()) return false;
        Progress &p = it->second;
        const int wt = p.knn ? kWindows * kTrials : 0;
        // the fastest trial of each setting (a slow one is noise: the first
        // call of a shape also allocates its workspace)
        double &best_ms =
            p.trial < wt ? p.ms_per_q[p.trial % kWindows] : p.ms_per_q[kWindows + (p.trial - wt) % kGrids];
        if (best_ms == 0.0 || ms_per_query < best_ms) best_ms = ms_per_query;
        p.trial++;
        if (p.knn && p.trial == wt) {
            p.best.window = 0;
            for (int c = 1; c < kWindows; c++)
                if (p.ms_per_q[c] < p.ms_per_q[p.best.window]) p.best.window = c;
        }
        if (p.trial < p.total()) return false;
        p.best.grid = 0;
        for (int c = 1; c < kGrids; c++)
            if (p.ms_per_q[kWindows + c] < p.ms_per_q[kWindows + p.best.grid]) p.best.grid = c;
        *done = p.best;
        keys.erase(it);
        last_tuning = false;
        return true;
    }
};

// Bump allocation over a fixed device region (the no-allocation entry
// point's scratch array): buffers are carved in order, 256-byte aligned, and
// the whole region is reused by the next call.
struct Arena {
    uint8_t *base = nullptr;
    size_t size = 0, used = 0;
    size_t left() const { return size > align(used) ? size - align(used) : 0; }
    static size_t align(size_t v) { return (v + 255) / 256 * 256; }
    void *take(size_t bytes)
    {
        const size_t at = align(used);
        if (at + bytes > size)
            fail(GTS_ENOMEM, "the no-allocation scratch (" + std::to_string(size) + " bytes) cannot hold this batch's "
                             "intermediate data; use a smaller batch");
        used = at + bytes;
        return base + at;
    }
};

// What a server batch sees of an index that keeps changing while it runs.
// Every update has an epoch (the index's counter after the update); a query
// admitted at epoch e sees the tree positions not deleted by updates of
// epoch <= e and the cache slots inserted, and not deleted, by them.  The
// batch reads the cache slots below cache_count only (later inserts go to
// higher slots); producers run on the tombstones of the earliest epoch of the
// batch, the kNN bounds on those of the latest, and each candidate is then
// checked against its own query's epoch.
struct SnapView {
    bool on = false;
    std::vector<uint32_t> qep;         // epoch of each query (caller order)
    int64_t cache_count = 0;
    uint32_t e_min = 0, e_max = 0;
};

struct QueryCtx {
    hipStream_t stream = nullptr;
    Arena *arena = nullptr;            // set: every workspace buffer is carved from it
    SnapView view;                     // on: the search follows these epochs (server batches)
    // graph mode (search plans, being recorded into a hipGraph): device
    // radius / k arrays, no host reads or synchronisation, fixed-capacity
    // buffers from the arena, device-side verification plan; failures are
    // flags in the device word gstatus
    bool graph = false;
    uint32_t *gstatus = nullptr;
    DevBuf ws[kWorkspaceSlots];        // grown on demand, reused across calls
    void *pin = nullptr;               // pinned host staging for small device-to-host reads
    size_t pin_bytes = 0;
    hipEvent_t ev[9] = {};
    bool timing = false;
    gts_stats stats{};
    LaunchTuner tuner;
    QueryCtx() = default;
    QueryCtx(const QueryCtx &) = delete;
    QueryCtx &operator=(const QueryCtx &) = delete;
    bool pin_fixed = false;            // the staging was sized at set-up and never grows
    // at least `bytes` of pinned host memory (grown, never shrunk)
    void *pinned(size_t bytes)
    {
        if (bytes > pin_bytes && pin_fixed) return nullptr;
        if (bytes > pin_bytes) {
            if (pin) (void)hipHostFree(pin);
            pin = nullptr;
            pin_bytes = 0;
            const size_t want = std::max<size_t>(bytes, (size_t)1 << 16);
            if (hipHostMalloc(&pin, want, hipHostMallocDefault) != hipSuccess) {
                pin = nullptr;
                return nullptr;
            }
            pin_bytes = want;
        }
        return pin;
    }
    ~QueryCtx()
    {
        for (auto &e : ev)
            if (e) (void)hipEventDestroy(e);
        if (pin) (void)hipHostFree(pin);
    }
};
// Tune-cache file: lines "key window grid" (indexes into LaunchTuner's
// tables); unreadable or malformed lines are ignored.
void tune_cache_load(gts_index *idx);
void tune_cache_store(gts_index *idx);
// Run f, turning exceptions into a status and this thread's error text (the
// wrapper of every C-ABI entry point).
gts_status run_guarded(const std::function<void()> &f);
// Release a result allocated by search.
void free_result(gts_result *r);
// Caller-owned device output of the no-allocation search: CSR offsets
// [nq + 1], ids and distances [capacity]; *total receives the answer count
// (also when it exceeds the capacity, which is an ENOMEM failure).
struct NoAllocOut {
    int64_t *offsets;
    int64_t *ids;
    void *dist;
    int64_t capacity;
    int64_t *total;
};
// Largest batch of the no-allocation search (its pinned staging is sized for
// it when the index is built).
constexpr int64_t kNoAllocMaxQueries = 2048;
// Pinned staging bytes a search of nq queries needs.
size_t staging_bytes(int64_t nq);
// Queries.  With na set, cx->arena must be set: every intermediate buffer
// comes from the arena, the answers go to na's buffers, and the call
// allocates no device or pinned memory.
void search(gts_index *idx, QueryCtx *cx, const gts_objects *Q, const float *radius, const int32_t *k,
            const gts_query_opts *opts, gts_result *out, const NoAllocOut *na = nullptr);
// Copy a user object set (host or device) into host memory with fresh ids
// starting at first_id; validates values and lengths.  angular: the rows are
// scaled to unit length (norm in double, rounded to float); a zero row has no
// direction and is an EINVAL error.
void read_objects(const gts_objects *o, int32_t metric, int32_t dim, int32_t max_strlen, HostObjects *out,
                  bool angular = false);
// Vector objects already on the device into rows of dp floats (dim rounded
// up to 4, zero padding) on the device, validated there (finite; angular:
// scaled to unit length, a zero row an EINVAL error).
void read_rows_device(const gts_objects *o, int32_t dim, bool angular, hipStream_t st, DevBuf *rows);

}  // namespace gts

// The opaque handle of the C ABI.
struct gts_index {
    hipStream_t stream = nullptr;
    gts::IndexData data;
    gts::CacheList cache;
    gts::HostObjects host;             // objects of the tree, in the order they were built from
    std::vector<int32_t> host_row;     // position -> row of `host`
    gts::HostObjects cache_host;       // objects of the cache list, by slot
    std::vector<uint8_t> h_tomb;       // host mirror of the tombstones
    std::vector<int64_t> pos_of_id;    // id -> tree position (-1: not in tree)
    std::vector<int64_t> slot_of_id;   // id -> cache slot (-1: not in cache)
    int64_t next_id = 0;
    uint32_t epoch = 0;                // updates applied so far (each insert or delete call: one)
    int64_t n_deleted_tree = 0;
    int64_t rebuilds = 0;
    double rebuild_ms = 0.0;
    int32_t num_pivots = 0, fanout = 0;
    // GTS_COSINE_F32: the index is an L2 index over unit vectors; distances
    // are reported as angles 2 asin(d / 2) and radii converted to chords
    bool angular = false;
    // GTS_L1_F32: the vector index under the Manhattan metric (no bf16 MFMA
    // tables; candidates from the float32 pivot table, float32 distances)
    bool l1 = false;
    gts_build_opts opts{};
    std::string tune_cache;            // tuned-settings file ("" = none)
    std::mutex tune_mu;                // guards `tuned` and the file
    std::map<std::string, gts::TuneSetting> tuned;   // finished settings by shape key
    // Byte alphabet of every string stored so far (EDIT): lut[b] is the code
    // of byte b, or arows - 1 for a byte never stored (such a byte in a query
    // matches nothing).  Codes only grow with inserts; nothing stored depends
    // on them, every match table is built at query time.
    bool alpha[256] = {};
    gts::DevBuf lut;                   // uint8 [256]
    gts::DevBuf upd_buf;               // upload space of delete batches (grown, reused)
    int32_t arows = 1;
    // the default query context (on `stream`)
    gts::QueryCtx ctx;
    // the no-allocation search's context (on `stream`; pinned staging made at build)
    gts::QueryCtx ctx_na;
};
