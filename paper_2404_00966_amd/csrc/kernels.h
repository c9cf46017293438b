// Host-callable launchers of the libgts.so kernels (all asynchronous on `st`).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace gts {
namespace k {

// L2 verification: queries with more than kVerifyBlockMin candidates are
// verified by a whole workgroup; the verification order takes them first
// (class 0), then the others by decreasing candidate count (classes 1..4),
// so the longest start first.
constexpr int kVerifyBlockMin = 512;
constexpr int kVerifyClasses = 5;
__host__ __device__ inline int verify_class(int64_t ns)
{
    return ns > kVerifyBlockMin ? 0 : ns > 256 ? 1 : ns > 128 ? 2 : ns > 64 ? 3 : 4;
}

// Slots of the device counters behind gts_stats.
enum {
    CNT_NODE_TESTS = 0,
    CNT_LEAF_PAIRS = 1,
    CNT_TILE_PAIRS = 2,
    CNT_VERIFIED = 3,
    CNT_BOUND_EVALS = 4,
    CNT_BOUND_VIOL = 5,    // rechecked L2 candidates whose exact distance left their bf16 interval (must stay 0)
    CNT_OWN_PAIRS = 6,     // (query, object) pairs of the surviving (query, leaf) pairs (batched)
    CNT_FILTER_OBJS = 7    // objects staged by the pivot-table object filters (one read per (leaf, tile) item)
};
constexpr int kCounters = 8;
// Each counter is striped over kStripes words a cache line apart: a
// workgroup adds to stripe blockIdx.x % kStripes, so thousands of
// workgroups do not queue on one address.  The host sums the stripes.
constexpr int kStripes = 64;
constexpr int kStripeStride = 16;                       // 16 x 8 bytes = one 128-byte line
constexpr int kCounterWords = kCounters * kStripes * kStripeStride;
__device__ __forceinline__ void count_add(unsigned long long *counters, int which, unsigned long long v)
{
    atomicAdd(&counters[((size_t)which * kStripes + blockIdx.x % kStripes) * kStripeStride], v);
}

// Raise the launch error left by the wrapper `name` (a bad grid or resource
// request), so that it surfaces at its own call and not at a later one.
void check_launch(const char *name);
// Raise a not-supported error naming `what` unless ok (a launcher's own
// precondition on its arguments).
void require(bool ok, const char *what);

// A (query, object) pair on its way to the answer.
//   pos >= 0 : candidate at tree position pos; val = float bits of an
//              estimate of the squared distance (L2 tile path) or 0.
//   pos <  0 : already verified; val = sort key (distance bits << 32 | id).
struct alignas(16) Cand {
    int32_t q;
    int32_t pos;
    uint64_t val;
};
static_assert(sizeof(Cand) == 16, "a candidate is one 16-byte record");

// Candidate slots are reserved with one 64-bit atomic add per wave.  Every
// attempt counts, also past the buffer's capacity (only slots below it are
// written), so the count that reaches the host is the number of candidates
// the group produced: more than the capacity means "split and run again".
// With 32 bits a group making 2^32 or more attempts would wrap and look as
// if it fit.
using CandCount = unsigned long long;

// ---- preparation (k_prep.hip) ---------------------------------------------
void rows_bf16(const float *X, int64_t rows_valid, int64_t rows_pad, int dim, int stride, int ksteps,
               uint16_t *frag, float *norm2, float *err, float pad_norm2, hipStream_t st);
// l1: Manhattan distances instead of Euclidean (the same summation order).
void dist_l2_pivots(const float *X, int64_t rows, const float *P, int m, int mpad, int stride, float *out,
                    int64_t s_piv, int64_t s_row, hipStream_t st, bool l1 = false);
void dist_edit_pivots_f32(const uint8_t *chars, const int64_t *off, int64_t rows, const uint8_t *pchars,
                          const int32_t *poff, int m, int mpad, float *out, int64_t s_piv, int64_t s_row,
                          const uint8_t *lut, int arows, hipStream_t st);
void build_peq(const uint8_t *chars, const int64_t *off, int64_t nq, const uint8_t *lut, int arows, uint64_t *peq,
               hipStream_t st);
void thresholds(const float *base, const float *QP, const int32_t *kq, int64_t nq, int mpad, int is_edit,
                float delta, float pt_max, float *T, float *thr, float *cut, hipStream_t st);
void fill_u32(uint32_t *p, int64_t n, uint32_t v, hipStream_t st);
// dst[at[i]] = val[i] for i < n (the changed words of a delete batch)
void scatter_u32(uint32_t *dst, const uint32_t *at, const uint32_t *val, int64_t n, hipStream_t st);
// bits[w] (w < words): bit b set iff position 32 w + b < n has del_ep <= e.
void tomb_bits(const uint32_t *del_ep, int64_t n, uint32_t e, uint32_t *bits, int64_t words, hipStream_t st);
// out[t] += sum over leaves l of popcount(mask[l][t]) * leaf_cnt[l] (the
// (query, object) pairs a tile's surviving leaves hold); out zeroed first.
void tile_pairs(const uint64_t *mask, int64_t n_leaves, int ntiles, const int32_t *leaf_cnt, unsigned long long *out,
                hipStream_t st);
// *bad |= 1 when a value among the first dim of each row is not finite.
void check_finite(float *X, int64_t rows, int dim, int stride, uint32_t *bad, hipStream_t st);
// Graph-replayed searches: per-query parameters from device arrays (bit 1 of
// *status on bad input) and the final status word (see gts_plan_* in gts.h).
void query_params(const float *radius, const int32_t *k, int64_t nq, bool angular, float *base, int32_t *kq,
                  uint32_t *status, hipStream_t st);
void plan_status(uint32_t *status, const uint32_t *bad_query, const unsigned long long *cand_count, int64_t cand_cap,
                 const int64_t *total, int64_t answer_cap, hipStream_t st);
// Rows scaled to unit length in place (norm in double, result rounded to
// float); a row with zero or non-finite norm becomes zero and sets *bad.
void normalize_rows(float *X, int64_t rows, int dim, int stride, uint32_t *bad, hipStream_t st);
void sum_pad(const float *a, const float *b, int64_t n, int64_t npad, float *out, hipStream_t st);

// ---- tree and candidates (k_search.hip) ------------------------------------
struct TreeView {
    const float *box_aos;      // [n_nodes][2*mpad]
    const float *box_lo;       // [mpad][n_nodes]
    const float *box_hi;       // [mpad][n_nodes]
    const int32_t *leaf_first; // [n_leaves]
    const int32_t *leaf_cnt;   // [n_leaves]
    int64_t n_nodes, n_leaves, leaf0;
    int fanout, levels, mpad;
};

// Node filtering at leaf granularity: leaf_mask[leaf][tile] (bit = query
// lane whose global-pivot distances the leaf's box admits) for every leaf.
void leaf_box(const TreeView &t, const float *QP, const float *thr, int64_t nq, int ntiles, uint64_t *leaf_mask,
              unsigned long long *counters, hipStream_t st);

// Greedy descent to each query's home leaf (smallest box gap per level);
// for kNN queries (k[q] > 0) also the k-th smallest exact distance over a
// window of at least max(k, win) consecutive tree positions starting at the
// home leaf (deleted positions skipped; +inf if fewer than k are live).
struct L2View {
    const float *X32;          // [npad][dp]
    const float *xn, *xe;      // [npad]
    const uint16_t *X16t;      // fragments
    int64_t n, npad;
    int dim, dp, ksteps;
};
struct EditView {
    const uint8_t *chars;      // leaf order
    const int32_t *soff;       // [n + 1]
    int64_t n;
    const uint8_t *lut;        // [256] byte -> alphabet code (rows-1: outside)
    int rows;                  // alphabet size + 1 (rows of a match table)
};
struct QueryL2 {
    const float *Q32;          // [nq][dp]
    const uint16_t *Q16t;      // fragments
    const float *qn, *qe;      // [nqpad]
};
struct QueryEdit {
    const uint8_t *chars;
    const int64_t *off;        // [nq + 1]
    const uint64_t *peq;       // [nq][rows][4] match tables
};

void bound_l2(const TreeView &t, const L2View &o, const QueryL2 &qv, const float *QP, const int32_t *kq,
              int64_t nq, const uint32_t *tomb, int win, float *tq, int32_t *home, hipStream_t st, bool l1 = false);
// piv/cell_leaf (may be null): a query with a pivot centre h takes its window
// from the first object of cell h instead of its home leaf.
void bound_edit(const TreeView &t, const EditView &o, const QueryEdit &qv, const float *QP, const int32_t *kq,
                int64_t nq, const uint32_t *tomb, int win, float *tq, int32_t *home, const int32_t *piv,
                const int32_t *cell_leaf, hipStream_t st);

// Slab x query-tile bf16 MFMA distances (persistent, work counter in `work`).
struct SlabView {
    const float *emax, *nmax;
    const int32_t *leaf_lo, *leaf_hi;
    int64_t n_slabs;
};
// tqe[q] = T[q] + e_q (true-distance bound plus the query's bf16 error),
// -inf on padding rows; valid for whole 64-query tiles.
// Sweep workspace: (tile, mask) pairs of active (slab, tile) combinations,
// capacity n_slabs * ntiles; items (slab, first pair, count, -), capacity
// n_slabs * ceil(ntiles / kItemTiles); counts[3] (pairs, items, work cursor).
constexpr int kSweepItemTiles = 32;
struct SweepWork {
    int32_t *pair_tile;
    uint64_t *pair_mask;
    int4 *items;
    uint32_t *counts;
};
// The sweep's work list from the leaf masks (resets w.counts).
void slab_items(const SlabView &s, const uint64_t *leaf_mask, int ntiles, const SweepWork &w, hipStream_t st);
void mfma_sweep(const L2View &o, const SlabView &s, const QueryL2 &qv, const float *tqe, int64_t nq, int ntiles,
                const uint32_t *tomb, const SweepWork &w, Cand *cands, CandCount *cand_count, int64_t cand_cap,
                unsigned long long *counters, int grid_blocks, hipStream_t st);

// Edit-distance object filtering over (leaf, tile) items: length and pivot
// lower bounds, wave-ballot compaction into candidates.
void edit_objfilter(const TreeView &t, const int32_t *items, const uint32_t *item_count, int64_t item_cap,
                    const uint64_t *leaf_mask, int ntiles, const float *QP, const float *thr, const int32_t *qlen,
                    int64_t nq, const uint8_t *PTa, const int32_t *soff, const uint32_t *tomb, Cand *cands,
                    CandCount *cand_count, int64_t cand_cap, unsigned long long *counters, hipStream_t st);

// ---- float32 L2 selection (k_filter32.hip) ---------------------------------
// (leaf, tile) pairs whose mask keeps a query, leaf-major, as int32 pairs.
void mask_items(const uint64_t *leaf_mask, int64_t n_leaves, int ntiles, int32_t *items, uint32_t *item_count,
                int64_t item_cap, hipStream_t st);
// Lemma 1 over the float32 pivot table PT[mpad][n] for every object of the
// listed (leaf, tile) items; candidates carry no estimate (val = 0).
void l2_objfilter(const TreeView &t, const int32_t *items, const uint32_t *item_count, int64_t item_cap,
                  const uint64_t *leaf_mask, int ntiles, const float *QP, const float *thr, int64_t nq, const float *PT,
                  int64_t n, const uint32_t *tomb, Cand *cands, CandCount *cand_count, int64_t cand_cap,
                  unsigned long long *counters, hipStream_t st);

// Brute-force scans of the cache list; they emit verified entries with
// d <= cut (L2) or d <= floor(base) (edit distance).  Slot s is seen by a
// query of epoch e iff ins_ep[s] <= e < del_ep[s]; e = qep[q], or e_now for
// every query when qep is null.  Edit distance: with cp set, Lemma 1 on the
// global pivots (cp: the slots' pivot distances, QP: the queries') skips
// slots before their distance.
struct CacheScan {
    const uint32_t *ids, *ins_ep, *del_ep;   // [count]
    const float *cp;                          // [count][mpad] (null: no pivot test)
    int64_t count;
    int m, mpad;
    const uint32_t *qep;                      // [nq] admission epochs (null: e_now)
    uint32_t e_now;
    const float *QP;                          // [nq][mpad]
};
void cache_scan_l2(const float *Q32, int64_t nq, int dp, const float *C32, const CacheScan &cs, const float *cut,
                   Cand *cands, CandCount *cand_count, int64_t cand_cap, bool angular, hipStream_t st,
                   bool l1 = false);
void cache_scan_edit(const QueryEdit &qv, const EditView &o, int64_t nq, const uint8_t *cchars, int cstride,
                     const int32_t *clen, const CacheScan &cs, const float *base, Cand *cands, CandCount *cand_count,
                     int64_t cand_cap, hipStream_t st);
// Largest distance from each leaf's first object to the leaf's objects.
void leaf_radius_edit(const EditView &o, const int32_t *leaf_first, const int32_t *leaf_cnt, int64_t n_leaves,
                      float *leafR, hipStream_t st);
// Farthest-first centres over n objects (input order): keys[0] holds the
// key of the first centre, keys[1..K] must be zero; on return centers[j] is
// centre j, mind[o] the (squared, for L2) distance of object o to its nearest
// centre and near[o] that centre's number.
void fft_centers_l2(const float *X, int64_t n, int dp, int K, uint64_t *keys, int32_t *centers, float *mind,
                    int32_t *near, hipStream_t st, bool l1 = false);
void fft_centers_edit(const uint8_t *chars, const int64_t *off, int64_t n, const uint8_t *lut, int arows, int K,
                      uint64_t *keys, int32_t *centers, float *mind, int32_t *near, hipStream_t st);
// ---- device steps of the L2 build (k_build.hip) ----
// dst row p <- src row perm[p] (rows of dp floats, dp a multiple of 4).
void gather_rows(const float *src, int dp, const int32_t *perm, int64_t n, float *dst, hipStream_t st);
// Pivot table [mpad][n] into the order perm (rows m..mpad-1 zero).
void gather_pt(const float *src, const int32_t *perm, int64_t n, int m, int mpad, float *dst, hipStream_t st);
// out[o] = squared float32 distance of row o to centre row C[cell[o * stride]].
void centre_dist(const float *X, int dp, int64_t n, const int32_t *cell, int stride, const float *C, float *out,
                 hipStream_t st, bool l1 = false);
// near[o] = number of the nearest of the K centre rows C [K][dp] (exact
// float32 distances, first of equals; l1: Manhattan).
void nearest_centre(const float *X, int dp, int64_t n, const float *C, int K, bool l1, int32_t *near, hipStream_t st);
// Leaf order: perm sorted by (rank[cell[o * stride]], cdist[o], o); key
// returns each position's cell rank.  tmp holds sort_pairs_bytes(n).
void cell_order(const float *cdist, const int32_t *cell, int stride, const int32_t *rank, int n_cells, int64_t n,
                uint32_t *key, int32_t *perm, void *tmp, size_t tmp_bytes, hipStream_t st);
// Node boxes from the leaf-order pivot table: box_aos [n_nodes][2 mpad]
// (lo then hi), box_lo / box_hi [mpad][n_nodes].
void node_boxes(const float *PT, int64_t n, int m, int mpad, const int32_t *leaf_first, const int32_t *leaf_cnt,
                int64_t n_leaves, int64_t leaf0, int64_t n_nodes, int F, int levels, float *box_aos, float *box_lo,
                float *box_hi, hipStream_t st);
// Per 256-row slab: largest bf16 rounding error and norm (with margins) and
// the first and last leaf overlapping it.
void slab_summary(const float *xn, const float *xe, int64_t n, const int32_t *leaf_first, int64_t n_leaves,
                  int64_t n_slabs, float *emax, float *nmax, int32_t *sl, int32_t *sh, hipStream_t st);
// Leaf pivots: per leaf the object nearest its mean (rows into PL32 [lpad][dp])
// and the largest distance from it (leafR, widened); cen: [n_leaves][dim]
// doubles of scratch.  Empty leaves and j >= n_leaves: zero row, R = -inf.
void leaf_pivots(const float *X32, int dp, int dim, const int32_t *leaf_first, const int32_t *leaf_cnt,
                 int64_t n_leaves, int64_t lpad, double *cen, float *PL32, float *leafR, hipStream_t st,
                 bool l1 = false);
// pln[j] = +inf for j >= n_leaves and empty leaves.
void mark_empty(const int32_t *leaf_cnt, int64_t n_leaves, int64_t lpad, float *pln, hipStream_t st);
// *out = max(*out, max x) over non-negative floats, as float bits.
void max_f32(const float *x, int64_t n, uint32_t *out, hipStream_t st);
// Cells (the clusters that order the leaves, in chain order): centre
// strings, covering radius, box over the global pivot distances and the
// string-length range of each.
struct CellView {
    const uint8_t *chars;      // centre strings
    const int32_t *off;        // [n + 1]
    const float *R;            // [n] max distance centre -> member (-inf: empty)
    const float *box;          // [n][2 * mpad]: lo[0..mpad), hi[0..mpad)
    const int32_t *len;        // [n][2]: shortest and longest member
    int64_t n;
    const uint8_t *dist;       // [n][n] centre-to-centre distances
    const int32_t *qg_off;     // [kQgramBuckets + 1]
    const int32_t *qg_cell;    // centres whose string holds a q-gram of each bucket
};
// q-gram buckets of the centre strings: a q-gram (kQgram consecutive bytes)
// hashes to one of kQgramBuckets buckets; each bucket lists the centres
// holding a q-gram of that bucket.  Only the choice of a query's pivot centre
// depends on it (by vote count), never an answer.
constexpr int kQgram = 8;
constexpr int kQgramBits = 16;
constexpr int kQgramBuckets = 1 << kQgramBits;
__host__ __device__ inline uint32_t qgram_bucket(const uint8_t *s)
{
    uint32_t h = 0;
    for (int u = 0; u < kQgram; u++) h = h * 0x9E3779B1u + (uint32_t)s[u] + 1u;
    return h >> (32 - kQgramBits);
}
// Pivot centre of each query: among the (up to) four centres sharing the most
// q-gram buckets with it, the nearest by exact edit distance; piv[q] = its
// chain rank (-1: no shared bucket) and pivd[q] = d(q, centre).  With it the
// cell test applies Lemma 1 with that centre as the pivot:
// d(q, o) >= |d(q, h) - d(h, c)| - R_c for every member o of cell c.
void edit_pivot(const EditView &o, const QueryEdit &qv, int64_t nq, const CellView &cv, int32_t *piv,
                int32_t *pivd, hipStream_t st);
// Passing cells kept per query; a query with more takes every cell.
constexpr int kQueryCells = 64;
// Cell test (Lemma 1 with each centre, with the query's pivot centre and
// with the global pivots) for nq queries in tiles of 64, position p holding
// query order[p] (order may be null: the identity); piv/pivd are indexed by
// query (piv may be null: no pivot centre).  qcnt[p] = number of passing
// cells, qcells[p][0..63] the first kQueryCells of them (in no particular
// order).
void edit_cell_test(const EditView &o, const QueryEdit &qv, const int32_t *qlen, const float *QP, int mpad,
                    const float *T, int64_t nq, int max_qlen, const CellView &cv, const int32_t *piv,
                    const int32_t *pivd, int32_t *qcells, int32_t *qcnt, unsigned long long *counters,
                    const int32_t *order, hipStream_t st);
// First (chain-order) passing cell of each position: n_cells when none
// passed, 0 when the list overflowed.
void first_cell(const int32_t *qcells, const int32_t *qcnt, int64_t n_cells, int64_t nq, int32_t *home,
                hipStream_t st);
// Leaf test (Lemma 1 with each leaf's first object as its pivot) for every
// (query, leaf of a cell on its list): zeroes and fills leaf_mask[leaf][tile]
// and lists the nonzero (leaf, tile) pairs.
void edit_leaf_ball(const EditView &o, const QueryEdit &qv, const int32_t *qlen, const int32_t *leaf_first,
                    const float *leafR, const int32_t *leaf_cell, const int32_t *cell_leaf, int64_t n_cells,
                    const int32_t *qcells, const int32_t *qcnt, const float *T, int64_t nq, int ntiles,
                    int max_qlen, uint64_t *leaf_mask, int32_t *items, uint32_t *item_count, int64_t item_cap,
                    int64_t n_leaves, hipStream_t st);

// ---- grouping, verification, output (k_final.hip) ---------------------------
// Admission epochs (qep non-null, indexed by the candidates' query): tree
// candidates with del_ep[pos] <= qep[q] are left out of the groups.
void group_hist(const Cand *c, const CandCount *count, int64_t cap, uint32_t *qcount, const uint32_t *del_ep,
                const uint32_t *qep, hipStream_t st);
void scan_u32(const uint32_t *in, int64_t n, int64_t *out, hipStream_t st);  // out[n+1]
// Writes only entries below grouped_cap (a larger candidate count is
// scattered again into a larger buffer).
void group_scatter(const Cand *c, const CandCount *count, int64_t cap, const int64_t *qoff, uint32_t *cursor,
                   Cand *grouped, int64_t grouped_cap, const uint32_t *del_ep, const uint32_t *qep, hipStream_t st);

struct VerifyArgs {
    const Cand *grouped;       // candidates grouped by query
    const int64_t *qoff;       // [nq + 1]
    const int64_t *big_off;    // [nq]: scratch offset (power-of-two run) or -1
    uint64_t *scratch;         // big-segment sort space
    const int32_t *kq;         // [nq] 0 = range
    const float *base;         // [nq] range radius or kNN bound
    const uint32_t *ids;       // [n] id per position
    int64_t nq;
    uint64_t *out_keys;        // same index space as grouped
    uint32_t *out_count;       // [nq]
    unsigned long long *counters;
    int angular;               // L2 on unit vectors: keys carry the angle 2 asin(d/2)
    int l1;                    // vectors under the Manhattan (L1) metric
};
// order: [nq] every query once, the n_blk queries with more than
// kVerifyBlockMin candidates first (a whole workgroup each), then the others
// (one wave each) in the order they should start; n_blk from the host, or
// read from *n_blk_dev when the order was made on the device.  ctr:
// kVerifyCursorWords words, zero before the launch (the work-queue cursors).
// est: the tree-position candidates carry bf16 estimates of d^2 (the bf16
// selection); without them every candidate is rechecked and kept for the
// final (distance, id) cut.
// check: count rechecked candidates whose float32 distance leaves their
// bf16 interval (CNT_BOUND_VIOL).
constexpr int kVerifyRun = 64;                  // consecutive wave-mode queries of one XCD queue
constexpr int kVerifyCursorStride = 32;         // words between the work-queue cursors (128 bytes)
constexpr int kVerifyCursorWords = 8 * kVerifyCursorStride;
void verify_l2(const VerifyArgs &a, const L2View &o, const QueryL2 &qv, float delta, const int32_t *order, int n_blk,
               bool est, bool check, hipStream_t st, bool l1, const int32_t *n_blk_dev, uint32_t *ctr);
// The verification plan made on the device, in two steps.  Counts: need
// [ng] (each query's power-of-two scratch run, 0 when its keys fit the LDS
// sort), need_off [ng + 1] (their scan; need_off[ng] the scratch words),
// cls [kVerifyPlanWords] (cleared here): the queries per verify_class, then
// the classes' cursors, then the largest candidate count.  Lists: big_off
// (-1 or the query's scratch run) and the verification order (queries by
// class; within a class in no fixed order), *n_blk (may be null) the
// workgroup count.
constexpr int kVerifyPlanWords = 2 * kVerifyClasses + 1;
void verify_plan_count(const int64_t *qoff, int64_t ng, int64_t sort_cap, uint32_t *need, int64_t *need_off,
                       uint32_t *cls, hipStream_t st);
void verify_plan_lists(const int64_t *qoff, int64_t ng, const uint32_t *need, const int64_t *need_off, uint32_t *cls,
                       int64_t *big_off, int32_t *order, int32_t *n_blk, hipStream_t st);
// band_only: every cutoff floor(base[q]) of the launch is at most 63.
void verify_edit(const VerifyArgs &a, const EditView &o, const QueryEdit &qv, bool band_only, hipStream_t st);

// cc[perm[i]] = out_count[i] (cc[i] without perm): answer counts in the
// caller's query order.
void perm_counts(const uint32_t *out_count, const int32_t *perm, int64_t nq, uint32_t *cc, hipStream_t st);
// Result in the caller's query order straight from the sorted keys: batch
// query i (caller query perm[i], or i without perm) writes its out_count[i]
// keys from out_keys[qoff[i]] to ids / dist at dst_off[caller query].
void emit_result(const uint64_t *out_keys, const int64_t *qoff, const uint32_t *out_count, const int32_t *perm,
                 const int64_t *dst_off, int64_t nq, int is_edit, int64_t *ids, float *dist_f, int32_t *dist_i,
                 hipStream_t st, int64_t cap = -1);

// CSR assembly: ids[res_off[q] + j] and dist from out_keys[qoff[q] + j].
void csr_write(const uint64_t *out_keys, const int64_t *qoff, const uint32_t *out_count, const int64_t *res_off,
               int64_t nq, int is_edit, int64_t *ids, float *dist_f, int32_t *dist_i, hipStream_t st);

// ---- leaf pivots (k_leaf.hip) -------------------------------------------------
constexpr int kNearLeaves = 8;   // nearest leaf pivots kept per query
void leaf_near(const uint16_t *PL16t, const float *pln, int64_t lpad, int ksteps, const uint16_t *Q16t, int64_t nq,
               int32_t *near, hipStream_t st);
// Every per-query array into the batch order in one launch: row i of each
// destination <- row perm[i] of its source (base, k, pivot distances of
// width mpad, float32 rows of width dp, nearest leaves of width nnear; a
// null source is skipped).
void permute_queries(const int32_t *perm, int64_t nq, const float *base_s, float *base_d, const int32_t *kq_s,
                     int32_t *kq_d, const float *qp_s, float *qp_d, int mpad, const float *q32_s, float *q32_d,
                     int dp, const int32_t *near_s, int32_t *near_d, int nnear, hipStream_t st);
// Stable sort of the queries by home (home[q * stride], keys in [0, n_keys)):
// perm[i] = query at position i (k_sort.hip).  keys may alias home when
// stride is 1.
size_t home_sort_bytes(int64_t nq, int64_t n_keys);
void home_sort(const int32_t *home, int stride, int64_t nq, int64_t n_keys, uint32_t *keys, uint32_t *keys_sorted,
               int32_t *perm, void *tmp, size_t tmp_bytes, hipStream_t st);
void leaf_ball(const uint16_t *PL16t, const float *pln, const float *ple, const float *leafR, int64_t n_leaves,
               int ksteps, const uint16_t *Q16t, const float *qn, const float *qe, const float *T, int64_t nq,
               int ntiles, uint64_t *leaf_mask, const int32_t *leaf_cnt, unsigned long long *counters,
               hipStream_t st);
// only_unbounded: skip the kNN queries whose tq is already finite (bounded
// by bound_mfma).
void bound_near(const int32_t *near, const int32_t *leaf_first, const int32_t *leaf_cnt, const float *X32, int dp,
                const float *Q32, const int32_t *kq, int64_t nq, const uint32_t *tomb, int target, float *tq,
                unsigned long long *counters, hipStream_t st, bool only_unbounded = false);
// kNN bound of every kNN query from bf16 MFMA estimates over a window of
// whole 16-row groups shared by its 16-query block (the groups of the
// block's nearest leaves): tq = the k-th smallest upper interval end, or
// +inf when the window holds fewer than k live objects or not the whole
// window bound_near would read with the same target.
void bound_mfma(const uint16_t *X16t, const float *xn, const float *xe, int64_t n, int ksteps, const int32_t *near,
                const int32_t *leaf_first, const int32_t *leaf_cnt, const uint16_t *Q16t, const float *qn,
                const float *qe, const int32_t *kq, int64_t nq, const uint32_t *tomb, int target, float *tq,
                unsigned long long *counters, hipStream_t st);
void gather_rows(const float *src, const int32_t *perm, int64_t rows, int dp, float *dst, hipStream_t st);
// Stable sort of n (key, value) pairs by the low `bits` bits of the keys, in
// place (least significant 8-bit digit first); tmp holds sort_pairs_bytes(n).
size_t sort_pairs_bytes(int64_t n);
void sort_pairs_u32(uint32_t *keys, int32_t *vals, int64_t n, int bits, void *tmp, size_t tmp_bytes, hipStream_t st);
void gather_i32(const int32_t *src, const int32_t *perm, int64_t rows, int width, int32_t *dst, hipStream_t st);
void gather_strings(const uint8_t *src, const int64_t *src_off, const int32_t *perm, int64_t n, const int64_t *dst_off,
                    uint8_t *dst, hipStream_t st);
void unpermute(const int64_t *src_off, const int64_t *dst_off, const int32_t *perm, int64_t nq, const int64_t *src_ids,
               const uint32_t *src_dist, int64_t *dst_ids, uint32_t *dst_dist, hipStream_t st);

// ---- plain one-query-per-workgroup path (k_plain.hip) -----------------------
struct PlainArgs {
    int64_t nq;
    const float *base;         // [nq] radius or kNN bound (distance units)
    const int32_t *kq;         // [nq]
    int32_t *frontier;         // [grid][2][n_leaves]
    int grid;
    const uint32_t *tomb;
    const uint32_t *ids;       // [n] id per position
    Cand *out;
    CandCount *out_count;     // 64-bit reservation counter (attempts may exceed 2^32)
    int64_t out_cap;
    unsigned long long *counters;
    float delta, pt_max;
    const float *leaf_piv32;   // [n_leaves][dp] leaf pivot vectors (L2; null: no leaf test)
    const float *leafR;        // [n_leaves] largest pivot distance in the leaf
    int angular;               // L2 on unit vectors: keys carry the angle 2 asin(d/2)
    int l1;                    // vectors under the Manhattan (L1) metric
};
void plain_l2(const TreeView &t, const L2View &o, const float *P32, int m, const float *PT, const float *Q32,
              const PlainArgs &a, hipStream_t st);
void plain_edit(const TreeView &t, const EditView &o, const uint8_t *pchars, const int32_t *poff, int m,
                const uint8_t *PTe, const QueryEdit &qv, const PlainArgs &a, hipStream_t st);

}  // namespace k
}  // namespace gts
