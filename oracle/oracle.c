/*
 * CPU oracle for GTS batched similarity search -- TEST INFRASTRUCTURE ONLY.
 *
 * Only the tests, the smoke check and the CPU-baseline leg of the benchmark
 * may load this library.  The GPU library neither includes nor links it, and
 * this file shares no code, header, table or helper with the GPU path.
 *
 * What it computes (all in double precision for L2, int32 for edit distance):
 *
 *  1. The metrics themselves (Sec. 3, problem statement):
 *       - Euclidean distance, direct-difference form, summed in index order;
 *       - Manhattan (L1) distance, summed in index order;
 *       - Levenshtein distance with unit-cost insertion, deletion and
 *         replacement (the paper's string examples), by the full
 *         Wagner-Fischer dynamic programme.
 *  2. Metric range query MRQ(q, r) = { o : d(q, o) <= r } (Definition 1) and
 *     metric kNN query MkNNQ(q, k) (Definition 2), by brute-force linear
 *     scan.  Definition 2 admits any k-set under ties; the oracle fixes the
 *     first min(k, n) objects in ascending (distance, id) order.
 *  3. A separate GTS-literal tree search following the paper's index and
 *     query algorithms (Sec. 4.2-4.3 and 5.1-5.2, Algorithms 1-5), with the readings
 *     stated at each function.  It must return exactly what 2 returns; the
 *     tests check that, which also checks the readings.
 *
 * Parity pins live in tests/test_oracle_pins.py.
 */
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Object sets                                                              */
/* ------------------------------------------------------------------------ */

enum { ORC_L2 = 1, ORC_EDIT = 2, ORC_ANGULAR = 3, ORC_L1 = 4 };

typedef struct {
    int32_t metric;          /* ORC_L2, ORC_EDIT, ORC_ANGULAR or ORC_L1      */
    int32_t dim;             /* L2: vector length                            */
    int64_t n;               /* number of objects                            */
    const float *vecs;       /* L2: [n][dim] row-major                       */
    const uint8_t *chars;    /* EDIT: concatenated bytes                     */
    const int64_t *offsets;  /* EDIT: [n + 1] string start offsets           */
    const int64_t *ids;      /* [n] external ids, or NULL for 0..n-1         */
} orc_set;

typedef struct {
    int64_t nq;
    int64_t *offsets;        /* [nq + 1]                                     */
    int64_t *ids;            /* [offsets[nq]]                                */
    double *dist;            /* [offsets[nq]]                                */
} orc_result;

static int64_t set_id(const orc_set *s, int64_t i) { return s->ids ? s->ids[i] : i; }

/* Threads of the brute-force loops (timing on a given core count; results
 * do not depend on it).  Returns the count now in force. */
int32_t orc_set_threads(int32_t n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
    return (int32_t)omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}

/* Euclidean distance: sqrt(sum_i (x_i - y_i)^2) with every step in double. */
double orc_l2(const float *x, const float *y, int32_t dim)
{
    double acc = 0.0;
    for (int32_t i = 0; i < dim; i++) {
        double diff = (double)x[i] - (double)y[i];
        acc += diff * diff;
    }
    return sqrt(acc);
}

/* Manhattan (L1) distance, the metric of the paper's colour-histogram data:
 * sum_i |x_i - y_i| with every step in double, summed in index order. */
double orc_l1(const float *x, const float *y, int32_t dim)
{
    double acc = 0.0;
    for (int32_t i = 0; i < dim; i++) acc += fabs((double)x[i] - (double)y[i]);
    return acc;
}

/* Angular distance, the metric of cosine similarity on directions: the angle
 * theta in [0, pi] between nonzero x and y, theta = arccos(x.y / (|x| |y|)).
 * With the unit vectors u = x/|x| and v = y/|y|, |u - v| = 2 sin(theta/2) and
 * |u + v| = 2 cos(theta/2), so theta = 2 atan2(|u - v|, |u + v|); every step
 * in double.  (The half-angle form keeps full relative precision for angles
 * near 0 and pi, where arccos of a rounded cosine does not.)  A zero vector
 * has no direction: the result is NaN. */
double orc_angular(const float *x, const float *y, int32_t dim)
{
    double nx = 0.0, ny = 0.0;
    for (int32_t i = 0; i < dim; i++) {
        nx += (double)x[i] * (double)x[i];
        ny += (double)y[i] * (double)y[i];
    }
    nx = sqrt(nx);
    ny = sqrt(ny);
    if (nx == 0.0 || ny == 0.0) return NAN;
    double dm = 0.0, dp = 0.0;
    for (int32_t i = 0; i < dim; i++) {
        const double u = (double)x[i] / nx, v = (double)y[i] / ny;
        dm += (u - v) * (u - v);
        dp += (u + v) * (u + v);
    }
    return 2.0 * atan2(sqrt(dm), sqrt(dp));
}

/* Levenshtein distance by the Wagner-Fischer table, kept as two rows.
 * D[i][j] = cost of turning a[0..i) into b[0..j):
 *   D[i][0] = i, D[0][j] = j,
 *   D[i][j] = min(D[i-1][j] + 1, D[i][j-1] + 1, D[i-1][j-1] + [a[i-1] != b[j-1]]). */
int32_t orc_edit(const uint8_t *a, int64_t la, const uint8_t *b, int64_t lb)
{
    int32_t *prev = (int32_t *)malloc(sizeof(int32_t) * (size_t)(lb + 1));
    int32_t *cur = (int32_t *)malloc(sizeof(int32_t) * (size_t)(lb + 1));
    for (int64_t j = 0; j <= lb; j++) prev[j] = (int32_t)j;
    for (int64_t i = 1; i <= la; i++) {
        cur[0] = (int32_t)i;
        for (int64_t j = 1; j <= lb; j++) {
            int32_t del = prev[j] + 1;
            int32_t ins = cur[j - 1] + 1;
            int32_t sub = prev[j - 1] + (a[i - 1] != b[j - 1] ? 1 : 0);
            int32_t best = del < ins ? del : ins;
            cur[j] = best < sub ? best : sub;
        }
        int32_t *t = prev; prev = cur; cur = t;
    }
    int32_t d = prev[lb];
    free(prev);
    free(cur);
    return d;
}

/* Distance between object i of set A and object j of set B (same metric). */
static double set_dist(const orc_set *A, int64_t i, const orc_set *B, int64_t j)
{
    if (A->metric == ORC_L2)
        return orc_l2(A->vecs + (size_t)i * A->dim, B->vecs + (size_t)j * B->dim, A->dim);
    if (A->metric == ORC_ANGULAR)
        return orc_angular(A->vecs + (size_t)i * A->dim, B->vecs + (size_t)j * B->dim, A->dim);
    if (A->metric == ORC_L1)
        return orc_l1(A->vecs + (size_t)i * A->dim, B->vecs + (size_t)j * B->dim, A->dim);
    return (double)orc_edit(A->chars + A->offsets[i], A->offsets[i + 1] - A->offsets[i],
                            B->chars + B->offsets[j], B->offsets[j + 1] - B->offsets[j]);
}

double orc_set_dist(const orc_set *A, int64_t i, const orc_set *B, int64_t j)
{
    return set_dist(A, i, B, j);
}

/* All |Q| x |O| distances (row per query); used for quantile radii. */
void orc_pair_distances(const orc_set *O, const orc_set *Q, double *out)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t q = 0; q < Q->n; q++)
        for (int64_t o = 0; o < O->n; o++)
            out[(size_t)q * O->n + o] = set_dist(Q, q, O, o);
}

/* ------------------------------------------------------------------------ */
/* Brute force (Definitions 1 and 2)                                        */
/* ------------------------------------------------------------------------ */

typedef struct { double d; int64_t id; } orc_pair;

static int pair_cmp(const void *x, const void *y)
{
    const orc_pair *a = (const orc_pair *)x, *b = (const orc_pair *)y;
    if (a->d < b->d) return -1;
    if (a->d > b->d) return 1;
    return (a->id > b->id) - (a->id < b->id);
}

/* Pack per-query pair lists into a CSR result (the lists are consumed). */
static void pack_result(int64_t nq, orc_pair **lists, int64_t *counts, orc_result *out)
{
    out->nq = nq;
    out->offsets = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nq + 1));
    out->offsets[0] = 0;
    for (int64_t q = 0; q < nq; q++) out->offsets[q + 1] = out->offsets[q] + counts[q];
    int64_t total = out->offsets[nq];
    out->ids = (int64_t *)malloc(sizeof(int64_t) * (size_t)(total > 0 ? total : 1));
    out->dist = (double *)malloc(sizeof(double) * (size_t)(total > 0 ? total : 1));
    for (int64_t q = 0; q < nq; q++) {
        for (int64_t t = 0; t < counts[q]; t++) {
            out->ids[out->offsets[q] + t] = lists[q][t].id;
            out->dist[out->offsets[q] + t] = lists[q][t].d;
        }
        free(lists[q]);
    }
}

void orc_result_free(orc_result *r)
{
    free(r->offsets);
    free(r->ids);
    free(r->dist);
    r->offsets = NULL; r->ids = NULL; r->dist = NULL; r->nq = 0;
}

/* MRQ(q, r) = { o in O : d(q, o) <= r } for every query, sorted by (d, id). */
int orc_range_bf(const orc_set *O, const orc_set *Q, const double *radius, orc_result *out)
{
    int64_t nq = Q->n;
    orc_pair **lists = (orc_pair **)calloc((size_t)(nq > 0 ? nq : 1), sizeof(orc_pair *));
    int64_t *counts = (int64_t *)calloc((size_t)(nq > 0 ? nq : 1), sizeof(int64_t));
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t q = 0; q < nq; q++) {
        int64_t cap = 16, cnt = 0;
        orc_pair *l = (orc_pair *)malloc(sizeof(orc_pair) * (size_t)cap);
        for (int64_t o = 0; o < O->n; o++) {
            double d = set_dist(Q, q, O, o);
            if (d <= radius[q]) {
                if (cnt == cap) { cap *= 2; l = (orc_pair *)realloc(l, sizeof(orc_pair) * (size_t)cap); }
                l[cnt].d = d; l[cnt].id = set_id(O, o); cnt++;
            }
        }
        qsort(l, (size_t)cnt, sizeof(orc_pair), pair_cmp);
        lists[q] = l; counts[q] = cnt;
    }
    pack_result(nq, lists, counts, out);
    free(lists); free(counts);
    return 0;
}

/* MkNNQ(q, k): the first min(k, n) objects in ascending (d, id) order. */
int orc_knn_bf(const orc_set *O, const orc_set *Q, const int32_t *k, orc_result *out)
{
    int64_t nq = Q->n;
    orc_pair **lists = (orc_pair **)calloc((size_t)(nq > 0 ? nq : 1), sizeof(orc_pair *));
    int64_t *counts = (int64_t *)calloc((size_t)(nq > 0 ? nq : 1), sizeof(int64_t));
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t q = 0; q < nq; q++) {
        orc_pair *l = (orc_pair *)malloc(sizeof(orc_pair) * (size_t)(O->n > 0 ? O->n : 1));
        for (int64_t o = 0; o < O->n; o++) { l[o].d = set_dist(Q, q, O, o); l[o].id = set_id(O, o); }
        qsort(l, (size_t)O->n, sizeof(orc_pair), pair_cmp);
        int64_t kk = k[q] < O->n ? k[q] : O->n;
        lists[q] = l; counts[q] = kk < 0 ? 0 : kk;
    }
    pack_result(nq, lists, counts, out);
    free(lists); free(counts);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* GTS-literal tree (Sec. 4.2-4.3, Algorithms 1-3)                          */
/* ------------------------------------------------------------------------ */

typedef struct {
    int64_t pivot;     /* object index of this node's pivot, -1 if none      */
    double min_dis;    /* min distance of the node's objects to the PARENT's  */
    double max_dis;    /* pivot (max_dis is the symmetric upper end)          */
    int64_t size;      /* number of objects in the node                      */
    int64_t pos;       /* start of the node's run in the table list (0-based)*/
} orc_node;

typedef struct {
    orc_set objs;      /* borrowed: arrays stay owned by the caller          */
    int32_t nc;        /* node capacity N_c                                   */
    int32_t h;         /* number of partitioning layers                      */
    int64_t nnodes;    /* (N_c^(h+1) - 1) / (N_c - 1)                         */
    orc_node *nodes;   /* full N_c-ary numbering, root = 0                    */
    int64_t *tl_obj;   /* table list: object index at each position           */
    double *tl_dis;    /* distance of that object to its leaf's parent pivot  */
} orc_gts;

/* Smallest e with nc^e >= x (that is, ceil(log_nc(x)) for x >= 1). */
static int32_t ceil_log(int64_t x, int32_t nc)
{
    int32_t e = 0;
    long double p = 1.0L;
    while (p < (long double)x) { p *= nc; e++; }
    return e;
}

/* Height rule of Sec. 4.2: max_h = ceil(log_Nc(|O| + 1)) - 1 and the tree is
 * built to h = max_h - 1 layers, which leaves the last level overfull.
 * (Algorithm 1 writes h = ceil(log_Nc(|O|+1)) - 1; the text's rule is the one
 * that reproduces the worked example of Fig. 3, with 3 levels for 10 objects
 * and N_c = 2.) */
int32_t orc_gts_height(int64_t n, int32_t nc)
{
    int32_t h = ceil_log(n + 1, nc) - 2;
    return h < 0 ? 0 : h;
}

static uint64_t splitmix64(uint64_t *s)
{
    uint64_t z = (*s += 0x9E3779B97F4A7C15ULL);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

typedef struct { double dis; int64_t id; int64_t obj; } orc_sortrec;

static int sortrec_cmp(const void *x, const void *y)
{
    const orc_sortrec *a = (const orc_sortrec *)x, *b = (const orc_sortrec *)y;
    if (a->dis < b->dis) return -1;
    if (a->dis > b->dis) return 1;
    return (a->id > b->id) - (a->id < b->id);
}

static int64_t node_parent(int64_t v, int32_t nc) { return (v - 1) / nc; }

/* Pivot mapping for one node (Algorithm 2): the pivot is chosen by
 * farthest-first traversal -- the root takes a seeded random object, every
 * other node takes the object whose minimum distance to the pivots already
 * chosen on its path from the root is largest (ties: lowest id).  Then every
 * object's distance to the pivot goes into tl_dis. */
static void map_node(orc_gts *g, int64_t v, uint64_t *rng)
{
    orc_node *N = &g->nodes[v];
    if (N->size == 0) { N->pivot = -1; return; }
    const orc_set *S = &g->objs;
    if (v == 0) {
        N->pivot = g->tl_obj[N->pos + (int64_t)(splitmix64(rng) % (uint64_t)N->size)];
    } else {
        int64_t anc[64]; int na = 0;
        for (int64_t a = node_parent(v, g->nc);; a = node_parent(a, g->nc)) {
            if (g->nodes[a].pivot >= 0) anc[na++] = g->nodes[a].pivot;
            if (a == 0) break;
        }
        int64_t best = -1; double best_d = -1.0; int64_t best_id = 0;
        for (int64_t t = 0; t < N->size; t++) {
            int64_t o = g->tl_obj[N->pos + t];
            double m = INFINITY;
            for (int i = 0; i < na; i++) {
                double d = set_dist(S, o, S, anc[i]);
                if (d < m) m = d;
            }
            int64_t id = set_id(S, o);
            if (m > best_d || (m == best_d && id < best_id)) { best = o; best_d = m; best_id = id; }
        }
        N->pivot = best;
    }
    for (int64_t t = 0; t < N->size; t++)
        g->tl_dis[N->pos + t] = set_dist(S, g->tl_obj[N->pos + t], S, N->pivot);
}

/* Objects partitioning for one node (Algorithm 3): order the node's objects
 * by distance to its pivot and hand them out in equal-count runs; the last
 * child takes the remainder.  The paper orders by the real-valued key
 * node + dis/(max+1); here the order is the (dis, id) pair directly, which is
 * the same order without the precision loss of packing both in one number.
 * Child j of node v is v*N_c + j + 1 (Eq. 1 with a 0-based root), starts at
 * pos + j*avg and records min_dis/max_dis as the first/last distance of its
 * run. */
static void partition_node(orc_gts *g, int64_t v)
{
    orc_node *N = &g->nodes[v];
    const orc_set *S = &g->objs;
    int64_t size = N->size;
    if (size > 0) {
        orc_sortrec *r = (orc_sortrec *)malloc(sizeof(orc_sortrec) * (size_t)size);
        for (int64_t t = 0; t < size; t++) {
            r[t].dis = g->tl_dis[N->pos + t];
            r[t].obj = g->tl_obj[N->pos + t];
            r[t].id = set_id(S, r[t].obj);
        }
        qsort(r, (size_t)size, sizeof(orc_sortrec), sortrec_cmp);
        for (int64_t t = 0; t < size; t++) {
            g->tl_obj[N->pos + t] = r[t].obj;
            g->tl_dis[N->pos + t] = r[t].dis;
        }
        free(r);
    }
    int64_t avg = size / g->nc;
    for (int32_t j = 0; j < g->nc; j++) {
        orc_node *C = &g->nodes[v * g->nc + j + 1];
        C->pos = N->pos + (int64_t)j * avg;
        C->size = (j < g->nc - 1) ? avg : size - avg * (g->nc - 1);
        C->pivot = -1;
        if (C->size > 0) {
            C->min_dis = g->tl_dis[C->pos];
            C->max_dis = g->tl_dis[C->pos + C->size - 1];
        } else {
            C->min_dis = INFINITY;
            C->max_dis = -INFINITY;
        }
    }
}

/* Index construction (Algorithm 1): layer by layer, map then partition every
 * node of the layer.  After the last layer tl_dis holds, for each object, its
 * distance to the pivot of its leaf's parent -- the one table the paper keeps. */
orc_gts *orc_gts_build(const orc_set *objs, int32_t nc, uint64_t seed)
{
    if (nc < 2) return NULL;
    orc_gts *g = (orc_gts *)calloc(1, sizeof(orc_gts));
    g->objs = *objs;
    g->nc = nc;
    g->h = orc_gts_height(objs->n, nc);
    int64_t nn = 1, lvl = 1;
    for (int32_t l = 0; l < g->h; l++) { lvl *= nc; nn += lvl; }
    g->nnodes = nn;
    g->nodes = (orc_node *)calloc((size_t)nn, sizeof(orc_node));
    g->tl_obj = (int64_t *)malloc(sizeof(int64_t) * (size_t)(objs->n > 0 ? objs->n : 1));
    g->tl_dis = (double *)calloc((size_t)(objs->n > 0 ? objs->n : 1), sizeof(double));
    for (int64_t i = 0; i < objs->n; i++) g->tl_obj[i] = i;
    g->nodes[0].size = objs->n;
    g->nodes[0].pos = 0;
    g->nodes[0].pivot = -1;
    g->nodes[0].min_dis = 0.0;
    g->nodes[0].max_dis = 0.0;
    uint64_t rng = seed;
    int64_t first = 0, count = 1;
    for (int32_t layer = 1; layer <= g->h; layer++) {
        for (int64_t v = first; v < first + count; v++) map_node(g, v, &rng);
        for (int64_t v = first; v < first + count; v++) partition_node(g, v);
        first = first * nc + 1;
        count *= nc;
    }
    return g;
}

void orc_gts_free(orc_gts *g)
{
    if (!g) return;
    free(g->nodes); free(g->tl_obj); free(g->tl_dis); free(g);
}

int32_t orc_gts_layers(const orc_gts *g) { return g->h; }
int64_t orc_gts_node_count(const orc_gts *g) { return g->nnodes; }

/* Node records and the table list, for structural checks. */
void orc_gts_nodes(const orc_gts *g, int64_t *pivot_id, int64_t *size, int64_t *pos,
                   double *min_dis, double *max_dis)
{
    for (int64_t v = 0; v < g->nnodes; v++) {
        pivot_id[v] = g->nodes[v].pivot >= 0 ? set_id(&g->objs, g->nodes[v].pivot) : -1;
        size[v] = g->nodes[v].size;
        pos[v] = g->nodes[v].pos;
        min_dis[v] = g->nodes[v].min_dis;
        max_dis[v] = g->nodes[v].max_dis;
    }
}

void orc_gts_table(const orc_gts *g, int64_t *obj_id, double *dis)
{
    for (int64_t i = 0; i < g->objs.n; i++) {
        obj_id[i] = set_id(&g->objs, g->tl_obj[i]);
        dis[i] = g->tl_dis[i];
    }
}

/* ------------------------------------------------------------------------ */
/* GTS-literal search (Algorithms 4 and 5)                                  */
/* ------------------------------------------------------------------------ */

/* One element of the intermediate table Q_Res: node N to search for query q;
 * delta is d(q, pivot of N's parent), carried so the leaf table (whose
 * distances are to that pivot) can apply Lemma 1 object by object. */
typedef struct { int64_t node; int64_t q; double delta; } orc_elem;

/* Per-query answer pool.  Range: every verified object within the radius.
 * kNN: the k smallest (d, id) pairs seen so far, as a max-heap, plus the
 * sorted ids of pivots already added (a pivot is a real object and may also
 * reappear in a leaf; it must be counted once). */
typedef struct {
    orc_pair *a; int64_t n, cap;
    int64_t *piv; int64_t npiv, cappiv;
} orc_pool;

typedef struct {
    const orc_gts *g;
    const orc_set *Q;
    int32_t mode;            /* 0 range, 1 kNN                                 */
    const double *radius;    /* range radii                                    */
    const int32_t *k;        /* kNN k                                          */
    int64_t budget;          /* size_GPU of Algorithm 4, in table elements     */
    int64_t *evals;          /* distance evaluations per query                 */
    orc_pool *pool;
} orc_search;

static void push_back(orc_pool *P, double d, int64_t id)
{
    if (P->n == P->cap) {
        P->cap = P->cap ? 2 * P->cap : 16;
        P->a = (orc_pair *)realloc(P->a, sizeof(orc_pair) * (size_t)P->cap);
    }
    P->a[P->n].d = d; P->a[P->n].id = id; P->n++;
}

/* max-heap on (d, id) */
static int pair_gt(const orc_pair *x, const orc_pair *y) { return pair_cmp(x, y) > 0; }

static void heap_offer(orc_pool *P, int64_t k, double d, int64_t id)
{
    orc_pair e = { d, id };
    if (k <= 0) return;
    if (P->n < k) {
        push_back(P, d, id);
        int64_t i = P->n - 1;
        while (i > 0) {
            int64_t p = (i - 1) / 2;
            if (!pair_gt(&P->a[i], &P->a[p])) break;
            orc_pair t = P->a[i]; P->a[i] = P->a[p]; P->a[p] = t; i = p;
        }
        return;
    }
    if (!pair_gt(&P->a[0], &e)) return;         /* not better than the k-th */
    P->a[0] = e;
    int64_t i = 0;
    for (;;) {
        int64_t l = 2 * i + 1, r = l + 1, m = i;
        if (l < P->n && pair_gt(&P->a[l], &P->a[m])) m = l;
        if (r < P->n && pair_gt(&P->a[r], &P->a[m])) m = r;
        if (m == i) break;
        orc_pair t = P->a[i]; P->a[i] = P->a[m]; P->a[m] = t; i = m;
    }
}

static int pivot_seen(orc_pool *P, int64_t id)
{
    int64_t lo = 0, hi = P->npiv;
    while (lo < hi) { int64_t mid = (lo + hi) / 2; if (P->piv[mid] < id) lo = mid + 1; else hi = mid; }
    return lo < P->npiv && P->piv[lo] == id;
}

static void pivot_mark(orc_pool *P, int64_t id)
{
    if (P->npiv == P->cappiv) {
        P->cappiv = P->cappiv ? 2 * P->cappiv : 16;
        P->piv = (int64_t *)realloc(P->piv, sizeof(int64_t) * (size_t)P->cappiv);
    }
    int64_t i = P->npiv++;
    while (i > 0 && P->piv[i - 1] > id) { P->piv[i] = P->piv[i - 1]; i--; }
    P->piv[i] = id;
}

/* kNN bound: the k-th smallest distance among the objects verified so far
 * (Algorithm 5 locates "the k-th distance" of each query; it has to be the
 * k-th smallest for Lemma 2 to be sound), +inf while fewer than k are known. */
static double search_radius(const orc_search *s, int64_t q)
{
    if (s->mode == 0) return s->radius[q];
    const orc_pool *P = &s->pool[q];
    return (s->k[q] > 0 && P->n >= s->k[q]) ? P->a[0].d : INFINITY;
}

/* Leaf verification: Lemma 1 on each object with its stored parent-pivot
 * distance (prune when |d(o,p) - d(q,p)| > radius), then the real distance. */
static void verify_leaf(orc_search *s, const orc_elem *e)
{
    const orc_gts *g = s->g;
    const orc_node *N = &g->nodes[e->node];
    orc_pool *P = &s->pool[e->q];
    for (int64_t t = 0; t < N->size; t++) {
        int64_t p = N->pos + t;
        double rad = search_radius(s, e->q);
        if (e->node != 0 && fabs(g->tl_dis[p] - e->delta) > rad) continue;
        int64_t o = g->tl_obj[p];
        int64_t id = set_id(&g->objs, o);
        if (s->mode == 1 && pivot_seen(P, id)) continue;   /* distance already known */
        double d = set_dist(s->Q, e->q, &g->objs, o);
        s->evals[e->q]++;
        if (s->mode == 0) {
            if (d <= rad) push_back(P, d, id);
        } else {
            heap_offer(P, s->k[e->q], d, id);
        }
    }
}

static void search_layer(orc_search *s, const orc_elem *E, int64_t ne, int32_t layer);

/* The body of the group loop of Algorithms 4/5 for one query group at one
 * layer: compute d(q, N.pivot) once per element, then keep child N' unless
 * the interval [N'.min_dis, N'.max_dis] of parent-pivot distances lies more
 * than the radius away from it -- the node form of Lemma 1 (Sec. 5.1 prunes on
 * d(q,p) + r < min_dis; the max_dis side is the symmetric case).  For kNN the
 * radius is the k-th distance after all of this layer's pivot distances have
 * joined the pool (Algorithm 5 sorts them and locates the k-th before it
 * prunes), and pruning is strict ">" so that an object tied with the k-th
 * distance survives for the (d, id) tie-break (Lemma 2 as printed prunes on
 * ">=", which could drop a tied object with a smaller id). */
static void expand_layer(orc_search *s, const orc_elem *E, int64_t ne, int32_t layer)
{
    const orc_gts *g = s->g;
    double *delta = (double *)malloc(sizeof(double) * (size_t)(ne > 0 ? ne : 1));
    for (int64_t i = 0; i < ne; i++) {
        const orc_node *N = &g->nodes[E[i].node];
        delta[i] = set_dist(s->Q, E[i].q, &g->objs, N->pivot);
        s->evals[E[i].q]++;
        if (s->mode == 1) {
            orc_pool *P = &s->pool[E[i].q];
            int64_t pid = set_id(&g->objs, N->pivot);
            if (!pivot_seen(P, pid)) {
                pivot_mark(P, pid);
                heap_offer(P, s->k[E[i].q], delta[i], pid);
            }
        }
    }
    orc_elem *next = (orc_elem *)malloc(sizeof(orc_elem) * (size_t)(ne * g->nc > 0 ? ne * g->nc : 1));
    int64_t nn = 0;
    for (int64_t i = 0; i < ne; i++) {
        double rad = search_radius(s, E[i].q);
        for (int32_t j = 0; j < g->nc; j++) {
            int64_t c = E[i].node * g->nc + j + 1;
            const orc_node *C = &g->nodes[c];
            if (C->size == 0) continue;
            double gap = C->min_dis - delta[i];
            if (delta[i] - C->max_dis > gap) gap = delta[i] - C->max_dis;
            if (gap > rad) continue;
            next[nn].node = c; next[nn].q = E[i].q; next[nn].delta = delta[i]; nn++;
        }
    }
    free(delta);
    search_layer(s, next, nn, layer + 1);
    free(next);
}

/* Range_Q / Knn_Q of Algorithms 4 and 5 on the elements E[0..ne) (nodes of
 * level `layer`, 1-based; elements of one query are contiguous).
 *
 * Two-stage processing: size_limit = budget / ((h - layer + 1) * N_c); when
 * the table is larger, the queries are split, in query order, into groups
 * whose elements fit (a query that alone exceeds the limit forms its own
 * group) and the groups run one after another. */
static void search_layer(orc_search *s, const orc_elem *E, int64_t ne, int32_t layer)
{
    const orc_gts *g = s->g;
    if (ne == 0) return;
    if (layer > g->h) {                         /* elements are leaves */
        for (int64_t i = 0; i < ne; i++) verify_leaf(s, &E[i]);
        return;
    }
    int64_t size_limit = s->budget / ((int64_t)(g->h - layer + 1) * g->nc);
    if (size_limit < 1) size_limit = 1;
    if (ne <= size_limit) { expand_layer(s, E, ne, layer); return; }
    int64_t a = 0;
    while (a < ne) {
        int64_t b = a + 1;
        while (b < ne && E[b].q == E[a].q) b++;            /* the first query */
        while (b < ne) {                                   /* more, if they fit */
            int64_t c = b + 1;
            while (c < ne && E[c].q == E[b].q) c++;
            if (c - a > size_limit) break;
            b = c;
        }
        expand_layer(s, E + a, b - a, layer);
        a = b;
    }
}

static int gts_search(const orc_gts *g, const orc_set *Q, int32_t mode, const double *radius,
                      const int32_t *k, int64_t budget, orc_result *out, int64_t *evals)
{
    int64_t nq = Q->n;
    orc_search s;
    memset(&s, 0, sizeof s);
    s.g = g; s.Q = Q; s.mode = mode; s.radius = radius; s.k = k;
    s.budget = budget > 0 ? budget : INT64_MAX / 4;
    s.evals = evals;
    size_t m = (size_t)(nq > 0 ? nq : 1);
    s.pool = (orc_pool *)calloc(m, sizeof(orc_pool));
    for (int64_t q = 0; q < nq; q++) evals[q] = 0;
    if (g->objs.n > 0 && nq > 0) {
        orc_elem *E = (orc_elem *)malloc(sizeof(orc_elem) * (size_t)nq);
        for (int64_t q = 0; q < nq; q++) { E[q].node = 0; E[q].q = q; E[q].delta = 0.0; }
        search_layer(&s, E, nq, 1);
        free(E);
    }
    orc_pair **lists = (orc_pair **)calloc(m, sizeof(orc_pair *));
    int64_t *counts = (int64_t *)calloc(m, sizeof(int64_t));
    for (int64_t q = 0; q < nq; q++) {
        orc_pool *P = &s.pool[q];
        qsort(P->a, (size_t)P->n, sizeof(orc_pair), pair_cmp);
        lists[q] = P->a ? P->a : (orc_pair *)malloc(sizeof(orc_pair));
        counts[q] = P->n;
        free(P->piv);
    }
    pack_result(nq, lists, counts, out);
    free(lists); free(counts); free(s.pool);
    return 0;
}

/* Batched MRQ (Algorithm 4).  `budget` is the intermediate-table capacity in
 * elements (<= 0: unlimited); it changes the grouping, never the answer. */
int orc_gts_range(const orc_gts *g, const orc_set *Q, const double *radius, int64_t budget,
                  orc_result *out, int64_t *evals)
{
    return gts_search(g, Q, 0, radius, NULL, budget, out, evals);
}

/* Batched MkNNQ (Algorithm 5), answering with the first min(k, n) objects in
 * (d, id) order. */
int orc_gts_knn(const orc_gts *g, const orc_set *Q, const int32_t *k, int64_t budget,
                orc_result *out, int64_t *evals)
{
    return gts_search(g, Q, 1, NULL, k, budget, out, evals);
}
