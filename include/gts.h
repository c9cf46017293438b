/*
 * gts.h -- C ABI of the MI355X batched metric-tree search library (libgts.so).
 *
 * The library answers the two similarity queries of the GTS paper (Zhu et
 * al., "GTS: GPU-based Tree Index for Fast Similarity Search", PACMMOD 2024)
 * over a pivot-based metric tree kept in GPU memory:
 *
 *   MRQ(q, r)   = { o in O : d(q, o) <= r }                    (Definition 1)
 *   MkNNQ(q, k) = k objects no farther from q than any other   (Definition 2)
 *
 * for the Euclidean, Manhattan and angular metrics on float32 vectors and
 * the Levenshtein (edit) metric on byte strings, with streamed insertions and
 * deletions (Sec. 4.4).
 *
 * Conventions for every call:
 *   - Plain pointers only.  Each gts_objects says whether its arrays live in
 *     host or device (HIP) memory; radius and k arrays are always host arrays.
 *   - Inputs are borrowed for the duration of the call; build and insert copy
 *     what they keep.  The caller owns a gts_index and releases it with
 *     gts_destroy; results are owned by the library until gts_result_free.
 *   - Every call returns a gts_status.  On failure the outputs are untouched
 *     and gts_last_error() describes the failure (thread-local text).
 *   - All GPU work of an index is ordered on the HIP stream given at build.
 *     An index is not re-entrant: calls on one index must not overlap
 *     (concurrent use goes through a gts_server).
 *   - Ties: answers are sorted by (distance, id) ascending, and a kNN answer
 *     is the first min(k, number of live objects) objects in that order --
 *     the paper's Definition 2 admits any such set; this fixes one.
 *   - Distances: L2 answers carry Euclidean (not squared) float32 distances
 *     computed directly from the float32 coordinates; edit answers carry
 *     exact int32 distances.  An L2 range answer holds the objects whose
 *     float32 distance is <= r.
 */
#ifndef GTS_H
#define GTS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t gts_status;
#define GTS_OK 0
#define GTS_EINVAL (-1)   /* bad argument: null pointer, size, NaN radius ... */
#define GTS_ENOMEM (-2)   /* device or host allocation failed, or the budget
                             cannot hold even one query's intermediate data */
#define GTS_EDEVICE (-3)  /* a HIP call failed (message carries its text)    */
#define GTS_ENOTSUP (-4)  /* valid request this build does not support       */

/* Metrics (Sec. 3: any metric; the paper evaluates L2 and edit distance). */
#define GTS_L2_F32 1      /* Euclidean distance on float32 vectors            */
#define GTS_EDIT_U8 2     /* Levenshtein distance, unit costs, on byte strings */
#define GTS_COSINE_F32 3  /* angular distance of cosine similarity: the angle
                             arccos(x.y / (|x| |y|)) in radians, in [0, pi],
                             between nonzero float32 vectors (directions)    */
#define GTS_L1_F32 4      /* Manhattan distance sum_i |x_i - y_i| on float32
                             vectors (the paper's colour histograms); always
                             selected on the float32 pivot table (no bf16)   */

/* Where an array lives. */
#define GTS_HOST 0
#define GTS_DEVICE 1

/* Query execution forms. */
#define GTS_MODE_BATCHED 0  /* whole batch through shared tiles (default)      */
#define GTS_MODE_PLAIN 1    /* one query per workgroup, every stage fused      */

/* Arithmetic of L2 candidate selection in the batched form (the paper fixes
 * no precision; answers are the same under both, the float32 distances of
 * the answers are computed the same way):
 *   GTS_BF16_GUARDED: bf16 MFMA tiles with float32 accumulation estimate
 *     d^2 for every (query, object) pair of the surviving leaves; a proven
 *     bound on the estimate's error decides which pairs cannot be answers,
 *     and only the others get a float32 direct-difference distance.
 *   GTS_FP32: Lemma 1 on the float32 pivot table (every object of the
 *     surviving leaves, all global pivots) selects the candidates, and every
 *     candidate gets its float32 direct-difference distance.
 * Edit distance is integer throughout and ignores the setting. */
#define GTS_PRECISION_DEFAULT 0  /* the index's setting (build: GTS_BF16_GUARDED) */
#define GTS_BF16_GUARDED 1
#define GTS_FP32 2

/* A set of objects (or queries).
 *   L2:   vecs = [n][dim] float32 row-major, finite values.
 *   EDIT: chars = concatenated bytes, offsets = [n + 1] int64 start offsets
 *         (offsets[0] = 0, non-decreasing); string i is
 *         chars[offsets[i] .. offsets[i+1]).  Lengths must not exceed the
 *         index's max_strlen (<= 255).
 *   location: GTS_HOST or GTS_DEVICE for all arrays of the set. */
typedef struct {
    int64_t n;
    int32_t dim;
    int32_t location;
    const float *vecs;
    const uint8_t *chars;
    const int64_t *offsets;
} gts_objects;

/* Index build options (all fields 0 -> defaults). */
typedef struct {
    uint64_t seed;           /* first-pivot choice of farthest-first traversal */
    int32_t leaf_size;       /* max objects per leaf; 0 = the paper's height
                                rule h = ceil(log_F(n + 1)) - 2 (Sec. 4.2)      */
    int32_t max_strlen;      /* EDIT: longest accepted string (default 255)    */
    int64_t cache_limit;     /* streamed inserts held in the cache list before
                                the index is rebuilt (Sec. 4.4); default 4096  */
    int64_t mem_budget_bytes;/* device bytes for a query batch's intermediate
                                data; 0 = 1/4 of free device memory            */
    int32_t precision;       /* GTS_BF16_GUARDED (0 = this) or GTS_FP32         */
    int32_t reserved0;       /* must be 0                                       */
    const char *tune_cache;  /* NULL, or a text file of tuned launch settings:
                                read at build, rewritten when the index's
                                default query context finishes tuning, keyed
                                by device, metric, dimension, pivots, fanout
                                and batch size (answers never depend on it)  */
} gts_build_opts;

/* Per-call query options (NULL -> defaults). */
typedef struct {
    int32_t mode;            /* GTS_MODE_BATCHED or GTS_MODE_PLAIN             */
    int32_t result_location; /* GTS_HOST or GTS_DEVICE; default: the queries'  */
    int64_t mem_budget_bytes;/* overrides the index's budget when > 0          */
    int32_t precision;       /* GTS_PRECISION_DEFAULT, GTS_BF16_GUARDED or
                                GTS_FP32 (batched L2; overrides the index's)   */
    int32_t flags;           /* GTS_QF_* bits (0: none)                         */
} gts_query_opts;

/* gts_query_opts.flags */
#define GTS_QF_CHECK_BOUND 1 /* L2, bf16 selection: test every rechecked
                                candidate's float32 distance against the
                                interval the proven bf16 error bound gave it
                                and count failures in gts_stats.
                                bound_violations (a self-check; answers do not
                                change, verification slows by about a third) */
#define GTS_QF_NO_PRUNE 2    /* L2 batched: a control without the tree -- every
                                (leaf, query) pair kept, so the selection tiles
                                cover every object for every query, as a dense
                                distance table would (kNN radii still come from
                                the nearest leaves' objects).  Same answers.  */

/* Answers in CSR form: the answer of query i is entries
 * offsets[i] .. offsets[i+1] of ids / dist.  Owned by the library. */
typedef struct {
    int64_t nq;
    int64_t total;
    int32_t location;        /* where offsets/ids/dist live                    */
    int32_t metric;
    int64_t *offsets;        /* [nq + 1]                                       */
    int64_t *ids;            /* [total] object ids                             */
    float *dist_f32;         /* [total] L2 distances (NULL for EDIT)           */
    int32_t *dist_i32;       /* [total] edit distances (NULL for L2)           */
    void *priv;              /* library bookkeeping; do not touch              */
} gts_result;

/* Work counters and stage times of the last query call on an index. */
typedef struct {
    int64_t nq;
    int64_t node_tests;      /* (query, node) box tests evaluated              */
    int64_t leaf_pairs;      /* surviving (query, leaf) pairs                   */
    int64_t tile_pairs;      /* (256-object slab, 16-query block) MFMA units    */
    int64_t candidates;      /* (query, object) pairs reaching verification    */
    int64_t verified;        /* exact metric evaluations                       */
    int64_t results;         /* answer entries                                 */
    double ms_total;         /* wall time of the call                          */
    double ms_stage[8];      /* device time per stage (GTS_STAGE_*)            */
    int64_t groups;          /* query groups run one after another (>1 when the
                                memory budget forced the two-stage split)      */
    int64_t bound_window;    /* L2 kNN: objects per query that bound the k-th
                                distance in this call (the tuned knob)         */
    int64_t tuning;          /* 1 while the query context is still trying
                                settings (answers are exact either way)        */
    int64_t bound_evals;     /* exact distances computed for the kNN bounds   */
    int64_t wide_queries;    /* queries whose candidates one whole workgroup
                                verified (L2: more than 1024; edit: more than
                                its LDS sort holds)                            */
    int64_t bound_violations;/* L2, bf16 selection with GTS_QF_CHECK_BOUND:
                                rechecked candidates whose float32 distance
                                fell outside the interval the proven error
                                bound gave them (0 unless the bound is wrong) */
    int64_t own_pairs;       /* batched: (query, object) pairs inside the
                                surviving (query, leaf) pairs -- the method's
                                own filtering work, before the tile rounding  */
    int64_t filter_objects;  /* objects read by the pivot-table object filters
                                (once per surviving (leaf, 64-query tile))     */
    int64_t sweep_grid_per_cu; /* L2 bf16 path: MFMA sweep workgroups per CU
                                in this call (the second tuned knob)           */
    int64_t group_retries;   /* query groups whose candidates overflowed the
                                memory budget and were split again (sized
                                from the attempt's counts)                     */
    int64_t max_query_candidates; /* largest candidate set of one query
                                (0 when a recorded graph ran the call)       */
} gts_stats;

#define GTS_STAGE_PREP 0     /* query -> pivot distances, query tiles          */
#define GTS_STAGE_BOUND 1    /* kNN radius bound                               */
#define GTS_STAGE_NODES 2    /* node filtering                                  */
#define GTS_STAGE_CANDS 3    /* object filtering / tile distances + compaction  */
/* GTS_STAGE_GROUP: grouping candidates by query, and the host's planning of
 * the verification after it; GTS_STAGE_VERIFY: from the verification launch. */
#define GTS_STAGE_GROUP 4    /* grouping candidates by query                    */
#define GTS_STAGE_VERIFY 5   /* exact verification, selection and sorting       */
#define GTS_STAGE_OUTPUT 6   /* CSR assembly                                    */
#define GTS_STAGE_PLAIN 7    /* the fused one-query-per-workgroup kernel        */

/* Index shape, for inspection and tests. */
typedef struct {
    int32_t metric, dim, num_pivots, fanout, levels, max_strlen;
    int64_t n_indexed;       /* objects in the tree (live or deleted)           */
    int64_t n_live;          /* live objects (tree + cache)                      */
    int64_t n_cache;         /* live objects in the cache list                   */
    int64_t n_nodes, n_leaves, n_slabs;
    int64_t rebuilds;        /* rebuilds triggered by the cache limit or by a
                                tree more than half deleted                     */
    int64_t device_bytes;    /* device memory held by the index                  */
    double rebuild_ms;       /* wall time spent in those rebuilds                */
    int64_t epoch;           /* updates applied so far (each insert or delete
                                call counts one)                                */
} gts_index_info;

typedef struct gts_index gts_index;

/* Build an index over `objs` (ids 0..n-1 in input order).
 * Follows the paper's construction (Sec. 4.3, Algorithms 1-3) with global
 * pivots: num_pivots pivots by farthest-first traversal (the first one
 * seeded) and every object's distance to every pivot in a pivot table; a
 * balanced tree of `fanout`-way nodes over leaves of near-equal size, the
 * objects ordered by cluster (farthest-first centres) so that leaves do not
 * straddle clusters.  Each node keeps the box of its objects' pivot
 * distances, each leaf a pivot of its own and its covering radius.
 * Requires num_pivots in [1, 32], fanout in [2, 64], n >= 1.
 * hip_stream: a hipStream_t (NULL = the null stream) used for all of the
 * index's GPU work.  On success *out receives the new index. */
gts_status gts_build_index(const gts_objects *objs, int32_t metric, int32_t num_pivots,
                           int32_t fanout, const gts_build_opts *opts, void *hip_stream,
                           gts_index **out);

/* Batched metric range query (Algorithm 4): answer i lists every live object
 * o with d(Q_i, o) <= radius[i].  radius: host array [Q->n] of finite values
 * >= 0 (for EDIT the integer part is used).  Q->n = 0 gives an empty answer.
 * The two-stage budget (Sec. 5.1) splits the batch into groups run one after
 * another when its intermediate data would exceed the budget; answers do not
 * depend on it.  GTS_ENOMEM if one query alone cannot fit. */
gts_status gts_range_query(gts_index *idx, const gts_objects *Q, const float *radius,
                           const gts_query_opts *opts, gts_result *out);

/* Batched metric kNN query (Algorithm 5 read as a range query whose radius is
 * bounded first, Sec. 5.2): answer i holds the min(k[i], live) live objects
 * nearest to Q_i in (distance, id) order.  k: host array [Q->n] of values
 * >= 1. */
gts_status gts_knn_query(gts_index *idx, const gts_objects *Q, const int32_t *k,
                         const gts_query_opts *opts, gts_result *out);

/* Mixed batch: query i is a kNN query when k != NULL and k[i] > 0, else a
 * range query with radius[i] (radius may be NULL only when every k[i] > 0).
 * Both kinds run through the same launches (Sec. 5: batched processing);
 * answers follow the conventions of gts_range_query / gts_knn_query. */
gts_status gts_search(gts_index *idx, const gts_objects *Q, const float *radius,
                      const int32_t *k, const gts_query_opts *opts, gts_result *out);

/* Streamed insertion (Sec. 4.4): the objects join the cache list, which every
 * query scans by brute force; when the cache holds more than cache_limit
 * objects the index is rebuilt over all live objects.  out_ids (host,
 * [objs->n], may be NULL) receives the new ids, which increase and are never
 * reused.  Ids stay below 2^31. */
gts_status gts_insert(gts_index *idx, const gts_objects *objs, int64_t *out_ids);

/* Streamed deletion (Sec. 4.4): an id in the cache list is removed from it;
 * an id in the tree is marked and skipped by every later query.  ids: host
 * array [n].  Unknown or already deleted ids are ignored; *n_deleted (may be
 * NULL) receives the number actually deleted. */
gts_status gts_delete(gts_index *idx, const int64_t *ids, int64_t n, int64_t *n_deleted);

/* Batch update (Sec. 4.4, batch updates): for bulk changes the index is
 * reconstructed directly instead of going through the cache list.  The ids
 * del_ids (host array [n_del]; unknown or deleted ids are ignored) are
 * deleted, the objects objs (may be NULL) are inserted with fresh ids
 * (out_ids, host [objs->n], may be NULL), and the index is rebuilt over every
 * live object, the cache list included (which ends empty).  *n_deleted (may
 * be NULL) receives the number of ids actually deleted. */
gts_status gts_update_batch(gts_index *idx, const gts_objects *objs, const int64_t *del_ids, int64_t n_del,
                            int64_t *out_ids, int64_t *n_deleted);

/* Cost model of a range query (Sec. 5.3, Eq. 2-3) over n objects with node
 * capacity (fanout) F:
 *   cost(F) = sum_{i=1..L} i^2 * ceil(F^i p^i / C) * log2(F)^2,
 * L = ceil(log_F n) layers, p = 1 - 2 sigma^2 / r^2 (the Chebyshev lower
 * bound of the probability that a pivot fails to prune an object; sigma^2
 * the variance of object-to-pivot distances, r the radius) clamped to
 * [0, 1], C the GPU's concurrency (threads in flight), each layer at least
 * one round.  NaN for n < 1, F < 2 or C <= 0.  Pure host arithmetic. */
double gts_cost_model(int64_t n, int32_t fanout, double sigma2, double radius, double concurrency);

/* The fanout in [2, 64] the cost model prefers for an object set (or a
 * sample of one; n is taken as objs->n): sigma^2 from the distances of up to
 * 2,048 seeded sample objects to one seeded sample pivot, radius r (for
 * GTS_COSINE_F32 an angle), concurrency C (<= 0: CUs x 2,048 of the current
 * device).  costs (may be NULL): [63] model cost of fanouts 2..64. */
gts_status gts_choose_fanout(const gts_objects *objs, int32_t metric, float radius, double concurrency,
                             int32_t *fanout, double *costs);

/* Copy a result into caller-provided buffers (same location kind as each
 * pointer: dst_location GTS_HOST or GTS_DEVICE); any pointer may be NULL. */
gts_status gts_result_copy(const gts_result *res, int32_t dst_location, int64_t *offsets,
                           int64_t *ids, void *dist);

/* Release a result's memory (safe on a zeroed or already freed result). */
gts_status gts_result_free(gts_result *res);

/* Release an index and all its device memory. */
gts_status gts_destroy(gts_index *idx);

/* Shape and counters of an index. */
gts_status gts_get_info(const gts_index *idx, gts_index_info *out);

/* Counters and stage times of the last query call on idx.  Stage times are
 * recorded only while stage timing is enabled (gts_set_timing). */
gts_status gts_get_stats(const gts_index *idx, gts_stats *out);

/* Enable (1) or disable (0) per-stage HIP-event timing on idx. */
gts_status gts_set_timing(gts_index *idx, int32_t enable);

/* Message of the last failure on this thread ("" if none). */
const char *gts_last_error(void);

/* ---- Search plans: a fixed-shape batch replayed as one HIP graph ----------
 * Batched processing (Sec. 5.1) of a query stream of a fixed shape: every
 * launch runs nq queries of a vector index (L2, L1 or angular) through the
 * whole batched pipeline -- pivot distances, home order, kNN bound, node and
 * object filters, candidate grouping, verification, answer assembly -- as
 * one hipGraph with fixed-capacity intermediate buffers and device-side
 * counts: no host synchronisation, allocation or host read inside a launch.
 *
 * gts_plan_create records the graph; the plan allocates its own
 * intermediate space (mem_budget_bytes from opts, or 1 GiB) and takes the
 * caller's device buffers in io, whose addresses the graph holds: they are
 * the caller's, and must stay allocated, at the same addresses, until the
 * plan is destroyed.  The caller writes queries [nq][dim] float32 (row-major),
 * radius [nq] (used where k == 0) and k [nq] (0: range query) before a
 * launch, and reads after it (in stream order): offsets [nq + 1] (CSR;
 * offsets[nq] is the number of answers, also when it exceeds the capacity),
 * ids and float distances [answer_capacity] (may be NULL when the capacity is
 * 0), and status (0: the launch's answers are complete; otherwise a sum of
 * GTS_PLAN_* flags, and the answers are not to be used).  gts_plan_launch
 * enqueues the graph on `hip_stream` (the index's own stream when NULL);
 * after an update or rebuild of the index it records the graph again first
 * (which waits for the device).  A plan is not re-entrant: launches of one
 * plan must not overlap, and the index must not be searched or updated while
 * one runs.  Edit-distance indexes: GTS_ENOTSUP. */
#define GTS_PLAN_BAD_INPUT 1       /* a negative k, or a negative or NaN radius */
#define GTS_PLAN_BAD_QUERY 2       /* a non-finite query value, or (angular) a zero query vector */
#define GTS_PLAN_CANDIDATES 4      /* the candidates exceed the plan's intermediate space */
#define GTS_PLAN_ANSWERS 8         /* the answers exceed answer_capacity */
typedef struct gts_plan gts_plan;
typedef struct gts_plan_io {
    const float *queries;          /* device, [nq][dim] */
    const float *radius;           /* device, [nq] */
    const int32_t *k;              /* device, [nq] */
    int64_t *offsets;              /* device, [nq + 1] */
    int64_t *ids;                  /* device, [answer_capacity] */
    float *dist;                   /* device, [answer_capacity] */
    int32_t *status;               /* device, [1] */
} gts_plan_io;
gts_status gts_plan_create(gts_index *idx, int64_t nq, int64_t answer_capacity, const gts_query_opts *opts,
                           const gts_plan_io *io, gts_plan **out);
gts_status gts_plan_launch(gts_plan *plan, void *hip_stream);
gts_status gts_plan_destroy(gts_plan *plan);

/* ---- No-allocation search --------------------------------------------------
 * For callers that cannot allocate memory during a query: code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation.
 *
 * The same answers as gts_search in the batched form (same conventions,
 * same kernels), but every intermediate buffer comes from one fixed device
 * array inside the library (GTS_NOALLOC_SCRATCH_BYTES, held by each GPU the
 * library runs on until the process ends), the pinned host staging was made
 * when the index was built, and the answers go to the caller's device
 * buffers: the call makes no hipMalloc, hipFree, hipHostMalloc or other
 * allocating runtime call.
 *   Q:            device queries (location GTS_DEVICE), at most
 *                 GTS_NOALLOC_MAX_QUERIES of them; radius / k as gts_search
 *                 (host arrays).
 *   opts:         may be NULL; mode must be GTS_MODE_BATCHED.
 *   out_offsets:  device int64 [Q->n + 1], CSR offsets of the answers.
 *   out_ids:      device int64 [out_capacity] object ids.
 *   out_dist:     device [out_capacity] float (L2) or int32 (EDIT) distances.
 *   out_total:    host int64: the number of answers, also on failure when
 *                 they exceed out_capacity (GTS_ENOMEM: retry with a larger
 *                 buffer).
 * GTS_ENOMEM also when the batch's intermediate data exceed the array (split
 * the batch).  Calls share the array: this process serialises them; calls
 * that overlap on one GPU from several threads wait for each other.  Stage
 * timing is not recorded and gts_get_stats reports the other calls. */
#define GTS_NOALLOC_SCRATCH_BYTES (128ll << 20)
#define GTS_NOALLOC_MAX_QUERIES 2048
gts_status gts_search_noalloc(gts_index *idx, const gts_objects *Q, const float *radius, const int32_t *k,
                              const gts_query_opts *opts, int64_t *out_offsets, int64_t *out_ids, void *out_dist,
                              int64_t out_capacity, int64_t *out_total);

/* ---- Serving: continuous batching over resident indexes -------------------
 *
 * A server owns worker threads over a set of built indexes (it does not own
 * the indexes; destroy the server first).  Requests are submitted one at a
 * time from any thread and complete asynchronously:
 *
 *   - Per index, requests take effect in submission order: a query sees
 *     exactly the inserts and deletes submitted to its index before it (its
 *     admission epoch).  An update waits for the index's batches in flight,
 *     runs alone, and the queries behind it wait for it.
 *   - Queries that queue up while others run are admitted together as the
 *     next batch (continuous batching: range and kNN requests of any k mix in
 *     one gts_search call), up to max_batch_queries, as soon as one of the
 *     index's lanes is free.  Each lane has its own HIP stream and query
 *     workspace, so batches of one index, and of different indexes, overlap
 *     on the device.  A batch's intermediate data is bounded by
 *     mem_budget_bytes through the two-stage split of gts_search.
 *   - Answers are the same as gts_search gives for the request alone on the
 *     index at its admission epoch. */
typedef struct gts_server gts_server;

#define GTS_REQ_RANGE 1
#define GTS_REQ_KNN 2
#define GTS_REQ_INSERT 3
#define GTS_REQ_DELETE 4

typedef struct {
    int32_t index;           /* position in the server's index list            */
    int32_t kind;            /* GTS_REQ_*                                      */
    gts_objects objects;     /* RANGE/KNN: the queries; INSERT: the new objects
                                (host or device; copied by gts_server_submit)  */
    float radius;            /* RANGE: radius of every query of the request    */
    int32_t k;               /* KNN: k of every query of the request (>= 1)    */
    const int64_t *ids;      /* DELETE: host array [n_ids] (copied)            */
    int64_t n_ids;
    uint64_t tag;            /* returned unchanged in the completion            */
} gts_request;

typedef struct {
    uint64_t ticket;         /* from gts_server_submit                          */
    uint64_t tag;
    int32_t kind;
    gts_status status;       /* GTS_OK, or why this request failed              */
    const char *error;       /* failure text ("" on success)                    */
    gts_result result;       /* RANGE/KNN: host CSR over the request's queries  */
    const int64_t *new_ids;  /* INSERT: [count] ids assigned                    */
    int64_t count;           /* INSERT: objects inserted; DELETE: ids deleted   */
    int64_t batch;           /* sequence number of the batch it ran in (-1: update) */
    double t_submit_ms;      /* steady-clock milliseconds                       */
    double t_start_ms;       /* its batch (or update) started                   */
    double t_done_ms;        /* answers were on the host                        */
    void *priv;
} gts_completion;

typedef struct {
    int32_t lanes_per_index; /* concurrent batches per index (default 2)        */
    int32_t max_batch_queries; /* queries per batch (default 16384)             */
    int64_t mem_budget_bytes;/* per batch (0: the index's budget / lanes)       */
    int32_t keep_results;    /* 0: record latencies and drop answers (no
                                completions are queued); default 1 when the
                                options pointer is NULL                         */
} gts_server_opts;

typedef struct {
    int64_t submitted, completed, failed;
    int64_t queries;         /* query objects answered                         */
    int64_t batches, updates;
    double mean_batch_queries;
    double p50_ms, p99_ms, max_ms; /* query requests: submit -> answers on host */
    double span_ms;          /* first submit -> last completion                 */
} gts_server_stats;

/* Start a server over n_indexes built indexes.  opts may be NULL. */
gts_status gts_server_create(gts_index *const *indexes, int32_t n_indexes, const gts_server_opts *opts,
                             gts_server **out);

/* Queue one request; *ticket (may be NULL) identifies its completion.
 * GTS_EINVAL for a malformed request (nothing is queued). */
gts_status gts_server_submit(gts_server *s, const gts_request *req, uint64_t *ticket);

/* Submit n requests at the given arrival times (milliseconds after the call
 * starts, non-decreasing), sleeping until each is due: an open-loop replay
 * of a trace.  tickets (may be NULL): [n]. */
gts_status gts_server_replay(gts_server *s, const gts_request *reqs, const double *arrival_ms, int64_t n,
                             uint64_t *tickets);

/* Take up to max completions, waiting up to wait_ms (0: do not wait, < 0:
 * until at least one is available or nothing is pending).  Each taken
 * completion must be released with gts_server_release. */
gts_status gts_server_poll(gts_server *s, gts_completion *out, int32_t max, int32_t wait_ms, int32_t *n_out);

/* Release a completion's memory. */
gts_status gts_server_release(gts_completion *c);

/* Wait until every submitted request has completed. */
gts_status gts_server_flush(gts_server *s);

/* Counters and latency percentiles since the server started. */
gts_status gts_server_get_stats(gts_server *s, gts_server_stats *out);

/* Finish every submitted request, stop the workers and free the server
 * (completions not yet polled are released). */
gts_status gts_server_destroy(gts_server *s);

#ifdef __cplusplus
}
#endif

#endif /* GTS_H */
