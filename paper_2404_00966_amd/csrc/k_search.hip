// Search kernels: node filtering, kNN radius bound, bf16 MFMA slab distances,
// edit-distance object filtering and the cache-list scan.
#include "dev_common.h"
#include "kernels.h"

namespace gts {
namespace k {


// Largest box gap of a query (pivot distances qp) to node `node`:
// max_i max(lo_i - qp_i, qp_i - hi_i).  A node whose gap exceeds the query's
// threshold holds no object within it (Lemma 1 applied to every pivot).
template <int MP>
__device__ __forceinline__ float box_gap(const float *__restrict__ box, int64_t node, const float *qp)
{
    const float *b = box + (size_t)node * 2 * MP;
    float g = -INFINITY;
#pragma unroll
    for (int i = 0; i < MP; i++) g = fmaxf(g, fmaxf(b[i] - qp[i], qp[i] - b[MP + i]));
    return g;
}

// ---------------------------------------------------------------------------
// Node filtering (the child test of Algorithms 4/5 with the global pivots,
// Lemma 1) down to the leaves, for every (64-query tile, leaf).  A node's box
// contains the boxes of its children (minima and maxima over the same
// objects), so a child can only pass where its parent passes: the walk from
// the root keeps exactly the leaves whose own box admits the query.  Here
// one ancestor level is tested first (the highest whose subtrees hold at
// most 64 leaves: the parents when the fanout is 16 or 32, the level six up
// for a binary tree) and the leaves below an ancestor that no query of the
// tile passes are not tested at all -- the same masks as the full walk,
// without its per-level launches.
//
// Lane = query: a workgroup is four 64-query tiles (one per wave, the pivot
// distances and threshold of its query in registers) and a range of leaves,
// whose boxes and parent boxes pass through LDS in chunks of 64 leaves and
// are read as broadcasts.  One ballot per tested node gives the tile's 64-bit
// query mask; lane j keeps the mask of the chunk's leaf j and stores it.
// Writes leaf_mask[leaf][tile] for every leaf and tile.  `group` is the
// number of leaves below one tested ancestor (a power of the fanout when the
// fanout divides 64: the chunk then holds whole subtrees), else 64 with no
// ancestor test; anc0 is the first node of the ancestors' level.
// ---------------------------------------------------------------------------
// A box staged as centres and half-widths (c[0..MP), r[0..MP)): the gap is
// max_i |q_i - c_i| - r_i, one subtraction fewer per pivot than from the
// bounds.  The halving and the subtractions each round once: the gap is
// within 4 u (|q| + the largest pivot distance) of the exact one, far inside
// the test's 2 delta (|q| + the largest pivot distance) margin, so no leaf
// the exact test keeps is dropped.
__device__ __forceinline__ void box_to_centre(float *lo_c, float *hi_r)
{
    const float lo = *lo_c, hi = *hi_r;
    float c = 0.f, r;
    if (!(lo <= hi)) r = -INFINITY;                              // empty: never entered
    else if (lo == -INFINITY || hi == INFINITY) r = INFINITY;    // unbounded: no constraint
    else {
        c = 0.5f * (lo + hi);
        r = 0.5f * (hi - lo);
    }
    *lo_c = c;
    *hi_r = r;
}

template <int MP>
__device__ __forceinline__ float box_gap_lds(const float *bx, const float *qp)
{
    float g = -INFINITY;
#pragma unroll
    for (int i = 0; i < MP; i++) g = fmaxf(g, fabsf(qp[i] - bx[i]) - bx[MP + i]);
    return g;
}

template <int MP>
__global__ __launch_bounds__(256) void k_leaf_box(const float *__restrict__ box, int64_t leaf0, int64_t n_leaves,
                                                  int group, bool parents, int64_t anc0,
                                                  const float *__restrict__ QP,
                                                  const float *__restrict__ thr, int64_t nq, int ntiles,
                                                  int64_t leaves_per_blk, int64_t n_split,
                                                  uint64_t *__restrict__ leaf_mask,
                                                  unsigned long long *__restrict__ counters)
{
    constexpr int kChunkVec = 64 * 2 * MP / 4;              // float4 per chunk of 64 boxes
    constexpr int kPerThread = (kChunkVec + 255) / 256;
    __shared__ float4 s_box4[kChunkVec];
    __shared__ float s_par[32 * 2 * MP];                    // ancestors of the chunk (group >= 2)
    const float *s_box = reinterpret_cast<const float *>(s_box4);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t tg = blockIdx.x / n_split, sp = blockIdx.x % n_split;
    const int tile = (int)(tg * 4 + wave);
    const bool live = tile < ntiles;                       // no early exit: barriers below
    const int64_t q = (int64_t)tile * 64 + lane;
    const bool qok = live && q < nq;
    float qp[MP];
#pragma unroll
    for (int i = 0; i < MP; i++) qp[i] = qok ? QP[(size_t)q * MP + i] : 0.f;
    const float th = qok ? thr[q] : -INFINITY;
    const int64_t lb = sp * leaves_per_blk;
    const int64_t le = min<int64_t>(n_leaves, lb + leaves_per_blk);
    long long tests = 0;
    for (int64_t c0 = lb; c0 < le; c0 += 64) {
        const int nl = (int)min<int64_t>(64, le - c0);
        const int np = (nl + group - 1) / group;
        __syncthreads();
        // all loads of the chunk are issued before the first is waited for
        const float4 *src = reinterpret_cast<const float4 *>(box + (size_t)(leaf0 + c0) * 2 * MP);
        const int nv = nl * 2 * MP / 4;
        float4 tv[kPerThread];
#pragma unroll
        for (int u = 0; u < kPerThread; u++) {
            const int i = u * 256 + (int)threadIdx.x;
            tv[u] = i < nv ? src[i] : make_float4(0.f, 0.f, 0.f, 0.f);
        }
        const int64_t par0 = anc0 + c0 / group;             // ancestor of the chunk's first leaf
#pragma unroll
        for (int u = 0; u < kPerThread; u++) {
            const int i = u * 256 + (int)threadIdx.x;
            if (i < kChunkVec) s_box4[i] = tv[u];
        }
        if (parents)
            for (int i = threadIdx.x; i < np * 2 * MP; i += blockDim.x) s_par[i] = box[(size_t)par0 * 2 * MP + i];
        __syncthreads();
        // bounds to centres and half-widths, in place
        float *sb = reinterpret_cast<float *>(s_box4);
        for (int i = threadIdx.x; i < nl * MP; i += blockDim.x) {
            const int j = i / MP, p = i - j * MP;
            box_to_centre(sb + j * 2 * MP + p, sb + j * 2 * MP + MP + p);
        }
        if (parents)
            for (int i = threadIdx.x; i < np * MP; i += blockDim.x) {
                const int j = i / MP, p = i - j * MP;
                box_to_centre(s_par + j * 2 * MP + p, s_par + j * 2 * MP + MP + p);
            }
        __syncthreads();
        uint64_t mine = 0;
        for (int pg = 0; pg < np; pg++) {
            const int j0 = pg * group, j1 = min(nl, j0 + group);
            if (parents) {
                tests++;
                if (!dev::ballot(box_gap_lds<MP>(s_par + pg * 2 * MP, qp) <= th)) continue;
            }
            tests += j1 - j0;
            for (int j = j0; j < j1; j++) {
                const uint64_t m = dev::ballot(box_gap_lds<MP>(s_box + j * 2 * MP, qp) <= th);
                mine = lane == j ? m : mine;
            }
        }
        if (live && lane < nl) leaf_mask[(size_t)(c0 + lane) * ntiles + tile] = mine;
    }
    if (live && lane == 0 && tests)
        count_add(counters, CNT_NODE_TESTS, (unsigned long long)min<int64_t>(64, nq - (int64_t)tile * 64) * (unsigned long long)tests);
}

void leaf_box(const TreeView &t, const float *QP, const float *thr, int64_t nq, int ntiles, uint64_t *leaf_mask,
              unsigned long long *counters, hipStream_t st)
{
    if (nq == 0 || t.n_leaves == 0) return;
    // about 2048 workgroups: leaf ranges of whole 64-leaf chunks
    const int64_t tgroups = (ntiles + 3) / 4, chunks = (t.n_leaves + 63) / 64;
    const int64_t per = std::max<int64_t>(1, chunks * tgroups / 2048);
    const int64_t lpb = 64 * per;
    const int64_t n_split = (t.n_leaves + lpb - 1) / lpb;
    const unsigned grid = (unsigned)(tgroups * n_split);
    // Leaves are tested below a passing ancestor: the one `up` levels above,
    // whose `group` = fanout^up leaves (at most 64, aligned with the 64-leaf
    // chunks when the fanout divides 64) are consecutive, so the chunk's
    // ancestors are consecutive nodes of their level, the first of them at
    // anc0.  A leaf's box lies inside every ancestor's box, so a query the
    // ancestor fails fails each of its leaves: the masks are those of the
    // leaf test alone.
    const bool parents = t.levels >= 1 && t.fanout >= 2 && 64 % t.fanout == 0;
    int group = 64, up = 0;
    if (parents) {
        group = t.fanout;
        up = 1;
        while (up < t.levels && (int64_t)group * t.fanout <= 64) {
            group *= t.fanout;
            up++;
        }
    }
    int64_t anc0 = t.leaf0;   // first node of the ancestors' level (heap order: parent(i) = (i - 1) / fanout)
    for (int u = 0; u < up; u++) anc0 = (anc0 - 1) / t.fanout;
#define LBX(MP)                                                                                                  \
    hipLaunchKernelGGL(k_leaf_box<MP>, dim3(grid), dim3(256), 0, st, t.box_aos, t.leaf0, t.n_leaves, group,     \
                       parents, anc0, QP, thr, nq, ntiles, lpb, n_split, leaf_mask, counters)
    if (t.mpad == 8) LBX(8);
    else if (t.mpad == 16) LBX(16);
    else LBX(32);
#undef LBX
    check_launch(__func__);
}

// ---------------------------------------------------------------------------
// kNN radius bound (the range-query strategy of Sec. 5.2: a kNN query is a
// range query once an upper bound of its k-th distance is known).  One
// 64-thread workgroup per query: descend greedily to the child with the
// smallest box gap, then take exact distances to a window of consecutive
// positions starting at that leaf; the k-th smallest of those is >= the true
// k-th distance.
// ---------------------------------------------------------------------------
constexpr int kWinMax = 1024;

template <int MP>
__device__ int64_t descend_home(const TreeView &t, const float *qp)
{
    const int lane = dev::lane_id();
    int64_t node = 0;
    for (int l = 1; l <= t.levels; l++) {
        int64_t child = node * t.fanout + 1 + lane;
        float g = INFINITY;
        if (lane < t.fanout) g = box_gap<MP>(t.box_aos, child, qp);
        float gmin = dev::wave_min(g);
        uint64_t who = dev::ballot(g == gmin);
        int best = who ? (__ffsll((long long)who) - 1) : 0;
        node = node * t.fanout + 1 + best;
    }
    return node - t.leaf0;
}

template <int MP, bool EDIT>
__global__ __launch_bounds__(64) void k_bound(TreeView t, L2View o, QueryL2 ql, EditView oe, QueryEdit qe,
                                              const float *__restrict__ QP, const int32_t *__restrict__ kq,
                                              int64_t nq, const uint32_t *__restrict__ tomb, int win,
                                              float *__restrict__ tq, int32_t *__restrict__ home,
                                              const int32_t *__restrict__ piv,
                                              const int32_t *__restrict__ cell_leaf, int l1)
{
    __shared__ float s_d[kWinMax];
    const int64_t q = blockIdx.x;
    if (q >= nq) return;
    const int lane = threadIdx.x;
    float qp[MP];
#pragma unroll
    for (int i = 0; i < MP; i++) qp[i] = QP[(size_t)q * MP + i];
    const int64_t leaf = descend_home<MP>(t, qp);
    if (lane == 0) home[q] = (int32_t)leaf;
    const int k = kq ? kq[q] : 0;
    if (k <= 0) return;
    const int64_t n = EDIT ? oe.n : o.n;
    int W = k > win ? k : win;
    if ((int64_t)W > n) W = (int)n;
    if (W > kWinMax || k > W) {           // no bound cheaper than a full scan
        if (lane == 0) tq[q] = INFINITY;
        return;
    }
    // the window starts at the home leaf, or (edit distance, when the query
    // has a pivot centre) is centred on that centre's cell: a family split
    // over two cells sits in neighbouring cells of the chain order, so a
    // small cell still gets its sibling's objects into the window
    int64_t a = t.leaf_first[leaf];
    if (piv && cell_leaf) {
        const int h = piv[q];
        if (h >= 0 && cell_leaf[2 * h] <= cell_leaf[2 * h + 1]) {
            const int l1 = cell_leaf[2 * h + 1];
            const int64_t c0 = t.leaf_first[cell_leaf[2 * h]], c1 = (int64_t)t.leaf_first[l1] + t.leaf_cnt[l1];
            a = (c0 + c1) / 2 - W / 2;
            if (a < 0) a = 0;
        }
    }
    if (a + W > n) a = n - W;
    const int Wp = dev::next_pow2(W);
    for (int j = lane; j < Wp; j += 64) {
        float d = INFINITY;
        if (j < W) {
            const int64_t p = a + j;
            const bool dead = (tomb[p >> 5] >> (p & 31)) & 1u;
            if (!dead) {
                if (!EDIT) {
                    const float4 *x = reinterpret_cast<const float4 *>(o.X32 + (size_t)p * o.dp);
                    const float4 *y = reinterpret_cast<const float4 *>(ql.Q32 + (size_t)q * o.dp);
                    float a0 = 0.f, a1 = 0.f, a2 = 0.f, a3 = 0.f;
                    if (l1) {
                        for (int c = 0; c < o.dp / 4; c++) {
                            const float4 u = x[c], v = y[c];
                            a0 = dev::dterm<true>(a0, u.x, v.x);
                            a1 = dev::dterm<true>(a1, u.y, v.y);
                            a2 = dev::dterm<true>(a2, u.z, v.z);
                            a3 = dev::dterm<true>(a3, u.w, v.w);
                        }
                    } else {
                        for (int c = 0; c < o.dp / 4; c++) {
                            const float4 u = x[c], v = y[c];
                            a0 = dev::dterm<false>(a0, u.x, v.x);
                            a1 = dev::dterm<false>(a1, u.y, v.y);
                            a2 = dev::dterm<false>(a2, u.z, v.z);
                            a3 = dev::dterm<false>(a3, u.w, v.w);
                        }
                    }
                    d = dev::dfinish_rt(l1 != 0, (a0 + a1) + (a2 + a3));
                } else {
                    const int32_t s0 = oe.soff[p];
                    const int tl = oe.soff[p + 1] - s0;
                    const int64_t qa = qe.off[q];
                    const int plen = (int)(qe.off[q + 1] - qa);
                    d = (float)dev::myers_any(qe.peq + (size_t)q * oe.rows * 4, plen, oe.chars + s0, tl, 1 << 30,
                                              oe.lut);
                }
            }
        }
        s_d[j] = d;
    }
    dev::bitonic_sort(s_d, Wp);
    if (lane == 0) tq[q] = s_d[k - 1];
}

void bound_l2(const TreeView &t, const L2View &o, const QueryL2 &qv, const float *QP, const int32_t *kq,
              int64_t nq, const uint32_t *tomb, int win, float *tq, int32_t *home, hipStream_t st, bool l1)
{
    if (nq == 0) return;
    EditView oe{};
    QueryEdit qe{};
#define BL(MP) \
    hipLaunchKernelGGL((k_bound<MP, false>), dim3((unsigned)nq), dim3(64), 0, st, t, o, qv, oe, qe, QP, kq, nq, tomb, win, tq, \
                       home, nullptr, nullptr, l1 ? 1 : 0)
    if (t.mpad == 8) BL(8);
    else if (t.mpad == 16) BL(16);
    else BL(32);
#undef BL
    check_launch(__func__);
}

void bound_edit(const TreeView &t, const EditView &o, const QueryEdit &qv, const float *QP, const int32_t *kq,
                int64_t nq, const uint32_t *tomb, int win, float *tq, int32_t *home, const int32_t *piv,
                const int32_t *cell_leaf, hipStream_t st)
{
    if (nq == 0) return;
    L2View ol{};
    QueryL2 ql{};
#define BE(MP) \
    hipLaunchKernelGGL((k_bound<MP, true>), dim3((unsigned)nq), dim3(64), 0, st, t, ol, ql, o, qv, QP, kq, nq, tomb, win, tq, \
                       home, piv, cell_leaf, 0)
    if (t.mpad == 8) BE(8);
    else if (t.mpad == 16) BE(16);
    else BE(32);
#undef BE
    check_launch(__func__);
}

// ---------------------------------------------------------------------------
// bf16 MFMA slab distances (L2 verification, first pass).
//
// Work item: one slab of 256 consecutive tree positions against a list of
// up to kItemTiles of its active query tiles (made by a pre-pass, so the
// persistent sweep never scans inactive tiles).  Each of the 4 waves keeps 64
// objects (4 row blocks of 16) as MFMA A fragments in registers for the whole
// item; query tiles (64 queries = 4 column blocks of 16) stream through LDS
// as B fragments, the next one copied while the current one computes.  With
// v_mfma_f32_16x16x32_bf16, lane l of the output holds objects 4*(l/16)+e
// (e = 0..3) of a row block and query l%16 of a column block.
//
// A pair is a candidate when its estimated squared distance
// qn + xn - 2 q.x does not exceed (T + e_q + e_slab)^2 + eps, where T bounds
// the true distance of any possible answer, e_q / e_slab bound the bf16
// rounding of the query / objects (||x16 - x|| <= e), and eps bounds the
// float32 error of the estimate.  So every answer is a candidate; the exact
// float32 distance is computed later for candidates only.
// ---------------------------------------------------------------------------
constexpr int kRowTiles = 4;  // 16-row MFMA blocks per wave: slab = 4 waves x 64 rows
static_assert(4 * 16 * kRowTiles == 256, "slab size must match the index layout");

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float floatx4_t __attribute__((ext_vector_type(4)));

__device__ __forceinline__ bf16x8_t as_bf16x8(uint4 v)
{
    bf16x8_t r;
    __builtin_memcpy(&r, &v, sizeof(r));
    return r;
}

// Pre-pass: the active query tiles of every slab (some query of the tile
// survives a leaf overlapping the slab) with the tile's union mask, written
// as (tile, mask) pairs, and work items of at most kItemTiles pairs of one
// slab.  One workgroup per kSlabsPerBlock slabs: count, reserve the pairs
// and items of all of them with one atomic each (not one per slab: the
// counters are shared by the whole grid), then fill.
constexpr int kItemTiles = kSweepItemTiles;

constexpr int kSlabsPerBlock = 16;

__global__ __launch_bounds__(256) void k_slab_items(const int32_t *__restrict__ slab_leaf_lo,
                                                    const int32_t *__restrict__ slab_leaf_hi, int64_t n_slabs,
                                                    const uint64_t *__restrict__ leaf_mask, int ntiles,
                                                    int32_t *__restrict__ pair_tile, uint64_t *__restrict__ pair_mask,
                                                    uint32_t *__restrict__ pair_count, int4 *__restrict__ items,
                                                    uint32_t *__restrict__ item_count)
{
    __shared__ uint32_t s_cnt[kSlabsPerBlock], s_pbase[kSlabsPerBlock], s_fill[kSlabsPerBlock];
    const int64_t slab0 = (int64_t)blockIdx.x * kSlabsPerBlock;
    const int ns = (int)min<int64_t>(kSlabsPerBlock, n_slabs - slab0);
    const int lane = threadIdx.x & 63;
    auto tile_mask = [&](int l_lo, int l_hi, int t) {
        uint64_t m = 0;
        for (int l = l_lo; l <= l_hi; l++) m |= leaf_mask[(size_t)l * ntiles + t];
        return m;
    };
    if (threadIdx.x < kSlabsPerBlock) {
        s_cnt[threadIdx.x] = 0;
        s_fill[threadIdx.x] = 0;
    }
    __syncthreads();
    for (int j = 0; j < ns; j++) {
        const int l_lo = slab_leaf_lo[slab0 + j], l_hi = slab_leaf_hi[slab0 + j];
        int cnt = 0;
        for (int t0 = 0; t0 < ntiles; t0 += blockDim.x) {
            const int t = t0 + (int)threadIdx.x;
            cnt += __popcll(dev::ballot(t < ntiles && tile_mask(l_lo, l_hi, t) != 0ull));
        }
        if (lane == 0 && cnt) atomicAdd(&s_cnt[j], (uint32_t)cnt);
    }
    __syncthreads();
    // one reservation of pairs and one of items for the block's slabs
    if (threadIdx.x == 0) {
        uint32_t total = 0, nit = 0;
        for (int j = 0; j < ns; j++) {
            total += s_cnt[j];
            nit += (s_cnt[j] + kItemTiles - 1) / kItemTiles;
        }
        const uint32_t pb = total ? atomicAdd(pair_count, total) : 0u;
        uint32_t ib = nit ? atomicAdd(item_count, nit) : 0u;
        uint32_t at = pb;
        for (int j = 0; j < ns; j++) {
            s_pbase[j] = at;
            const int c = (int)s_cnt[j];
            for (int k = 0; k * kItemTiles < c; k++)
                items[ib++] = make_int4((int)(slab0 + j), (int)(at + k * kItemTiles), min(kItemTiles, c - k * kItemTiles), 0);
            at += (uint32_t)c;
        }
    }
    __syncthreads();
    for (int j = 0; j < ns; j++) {
        if (s_cnt[j] == 0) continue;
        const int l_lo = slab_leaf_lo[slab0 + j], l_hi = slab_leaf_hi[slab0 + j];
        for (int t0 = 0; t0 < ntiles; t0 += blockDim.x) {
            const int t = t0 + (int)threadIdx.x;
            const uint64_t m = t < ntiles ? tile_mask(l_lo, l_hi, t) : 0ull;
            const uint64_t b = dev::ballot(m != 0ull);
            uint32_t at = 0;
            if (lane == 0 && b) at = atomicAdd(&s_fill[j], (uint32_t)__popcll(b));
            at = __shfl(at, 0, 64);
            if (m) {
                const uint32_t idx = s_pbase[j] + at + (uint32_t)dev::lanes_below(b);
                pair_tile[idx] = t;
                pair_mask[idx] = m;
            }
        }
    }
}

template <int KS, int RT>
__global__ __launch_bounds__(256, 2) void k_mfma_sweep(
    const uint4 *__restrict__ X16t, const float *__restrict__ xn, const uint4 *__restrict__ Q16t,
    const float *__restrict__ qn, const float *__restrict__ tqe, int64_t nq, const float *__restrict__ slab_emax,
    const float *__restrict__ slab_nmax, int64_t n, const uint32_t *__restrict__ tomb,
    const int32_t *__restrict__ pair_tile, const uint64_t *__restrict__ pair_mask, const int4 *__restrict__ items,
    const uint32_t *__restrict__ item_count, uint32_t *__restrict__ work, Cand *__restrict__ cands,
    CandCount *__restrict__ cand_count, int64_t cand_cap, float eps_a, float eps_b, float eps_c,
    unsigned long long *__restrict__ counters)
{
    constexpr int kRowsPerWave = 16 * RT;
    constexpr int kSlabRows = 4 * kRowsPerWave;
    constexpr int kTileFrag = 4 * KS * 64;           // uint4 fragments of one 64-query tile
    constexpr int kPer = kTileFrag / 256;            // fragments staged per thread
    constexpr int kCandBuf = 256;                    // per-wave candidate buffer
    // LDS: two staging buffers of one query tile (B fragments, T + e_q and
    // ||q16||^2 per query) and a candidate buffer per wave
    __shared__ uint4 s_b[2][kTileFrag];
    __shared__ float s_t[2][64], s_qn[2][64];
    __shared__ Cand s_cand[4][kCandBuf];
    __shared__ int4 s_item;
    const int wave = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    const int col = lane & 15;
    const int rgrp = lane >> 4;
    const int64_t n_items = *item_count;
    int64_t cur_slab = -1;
    uint4 A[RT][KS];
    float xr[RT][4];
    uint32_t live16 = 0;
    long long units = 0;
    Cand *cbuf = s_cand[wave];
    int nb = 0;   // buffered candidates of this wave (wave-uniform)
    auto flush = [&]() {
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        CandCount base = 0;
        if (lane == 0) base = atomicAdd(cand_count, (CandCount)nb);
        base = __shfl(base, 0, 64);
        // whole 16-byte records (one dwordx4 store per lane), so the flushed
        // run is written as full lines
        const uint4 *src = reinterpret_cast<const uint4 *>(cbuf);
        uint4 *dst = reinterpret_cast<uint4 *>(cands);
        for (int i = lane; i < nb; i += 64) {
            const int64_t idx = (int64_t)base + i;
            if (idx < cand_cap) dst[idx] = src[i];
        }
        __builtin_amdgcn_wave_barrier();
        nb = 0;
    };
    // query tile t through registers into LDS buffer b: every wave fetches
    // kPer 1 KB runs of fragments, waves 0 and 1 the two 256-byte parameter
    // rows.  The fetch of the next tile is issued before the current one
    // computes and written to LDS after it (plain loads: the LDS reads of the
    // current tile never wait on them).
    uint4 rs[kPer];
    float rt = 0.f, rq = 0.f;
    auto fetch = [&](int t) __attribute__((always_inline)) {
        const uint4 *src = Q16t + (int64_t)t * kTileFrag;
#pragma unroll
        for (int j = 0; j < kPer; j++) rs[j] = src[256 * j + threadIdx.x];
        if (wave == 0) rt = tqe[(int64_t)t * 64 + lane];
        if (wave == 1) rq = qn[(int64_t)t * 64 + lane];
    };
    auto put = [&](int b) __attribute__((always_inline)) {
#pragma unroll
        for (int j = 0; j < kPer; j++) s_b[b][256 * j + threadIdx.x] = rs[j];
        if (wave == 0) s_t[b][lane] = rt;
        if (wave == 1) s_qn[b][lane] = rq;
    };
    for (;;) {
        if (threadIdx.x == 0) {
            const uint32_t it = atomicAdd(work, 1u);
            s_item = it < n_items ? items[it] : make_int4(-1, 0, 0, 0);
        }
        __syncthreads();
        const int4 item = s_item;
        if (item.x < 0) break;
        const int64_t slab = item.x;
        const int p0 = item.y, ntl = item.z;
        const int64_t row0 = slab * kSlabRows + wave * kRowsPerWave;
        if (slab != cur_slab) {
            cur_slab = slab;
            const int64_t g0 = row0 >> 4;
#pragma unroll
            for (int r = 0; r < RT; r++)
#pragma unroll
                for (int s = 0; s < KS; s++) A[r][s] = X16t[((g0 + r) * KS + s) * 64 + lane];
#pragma unroll
            for (int r = 0; r < RT; r++)
#pragma unroll
                for (int e = 0; e < 4; e++) xr[r][e] = -0.5f * xn[row0 + 16 * r + 4 * rgrp + e];
            // this lane's 16 rows that are real, live objects (the wave's 64
            // rows span two tombstone words)
            const int64_t wd = row0 >> 5, nwords = (n + 31) >> 5;
            const uint32_t tw0 = wd < nwords ? tomb[wd] : ~0u, tw1 = wd + 1 < nwords ? tomb[wd + 1] : ~0u;
            live16 = 0;
#pragma unroll
            for (int r = 0; r < RT; r++)
#pragma unroll
                for (int e = 0; e < 4; e++) {
                    const int lr = 16 * r + 4 * rgrp + e;
                    const bool dead = ((lr < 32 ? tw0 >> lr : tw1 >> (lr - 32)) & 1u) || row0 + lr >= n;
                    live16 |= (dead ? 0u : 1u) << (4 * r + e);
                }
        }
        const float emax = slab_emax[slab];
        const float nmax = slab_nmax[slab];
        // the item's (tile, query mask) list in registers, lane j holding pair j
        const int my_tile = lane < ntl ? pair_tile[p0 + lane] : 0;
        const uint64_t my_mask = lane < ntl ? pair_mask[p0 + lane] : 0ull;
        fetch(__shfl(my_tile, 0, 64));
        put(0);
        __syncthreads();
        for (int it = 0; it < ntl; it++) {
            const int buf = it & 1;
            const int t = __shfl(my_tile, it, 64);
            const uint64_t mask = ((uint64_t)(uint32_t)__shfl((int)(uint32_t)(my_mask >> 32), it, 64) << 32) |
                                  (uint32_t)__shfl((int)(uint32_t)my_mask, it, 64);
            const bool more = it + 1 < ntl;
            if (more) fetch(__shfl(my_tile, it + 1, 64));   // lands while this tile computes
#pragma unroll 1
            for (int c = 0; c < 4; c++) {
                const uint32_t cm = (uint32_t)(mask >> (16 * c)) & 0xffffu;
                if (!cm) continue;
                units++;
                const int64_t q = (int64_t)t * 64 + 16 * c + col;
                float th = -INFINITY;
                const float qnn = s_qn[buf][16 * c + col];
                if (((cm >> col) & 1u) && q < nq) {
                    const float tq = s_t[buf][16 * c + col] + emax;
                    const float T2 = tq * tq;
                    const float eps = eps_a * (qnn + nmax * nmax) + eps_b * sqrtf(qnn) * nmax + eps_c * T2;
                    th = T2 + eps - qnn;
                }
                uint4 B[KS];
#pragma unroll
                for (int s = 0; s < KS; s++) B[s] = s_b[buf][(c * KS + s) * 64 + lane];
                // the accumulators start at -||x||^2 / 2, so the MFMA leaves
                // a = q.x - ||x||^2 / 2 and the test below is one compare:
                // xn - 2 q.x <= th  <=>  a >= -th / 2 (both scalings exact)
                floatx4_t acc[RT];
#pragma unroll
                for (int r = 0; r < RT; r++) acc[r] = floatx4_t{xr[r][0], xr[r][1], xr[r][2], xr[r][3]};
#pragma unroll
                for (int s = 0; s < KS; s++)
#pragma unroll
                    for (int r = 0; r < RT; r++)
                        acc[r] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(A[r][s]), as_bf16x8(B[s]), acc[r],
                                                                          0, 0, 0);
                // candidate test: xn - 2 q.x <= (T + e_q + e_slab)^2 + eps - qn;
                // one ballot per output element (a compare into a scalar mask),
                // the per-lane bits only when some pair passes
                const float thh = -0.5f * th;
                uint64_t anyp = 0;
#pragma unroll
                for (int r = 0; r < RT; r++)
#pragma unroll
                    for (int e = 0; e < 4; e++) anyp |= dev::ballot(acc[r][e] >= thh);
                if (anyp) {
                    uint32_t pm = 0;
#pragma unroll
                    for (int r = 0; r < RT; r++)
#pragma unroll
                        for (int e = 0; e < 4; e++) pm |= (acc[r][e] >= thh ? 1u : 0u) << (4 * r + e);
                    // drop padding rows and deleted objects, then compact into
                    // the wave's buffer (flushed with one atomic when full)
                    pm &= live16;
                    const int cnt = __popc(pm);
                    int tot;
                    const int off = dev::wave_excl_scan(cnt, &tot);
                    if (nb + tot > kCandBuf) flush();
                    if (tot > kCandBuf) {
                        // more than a buffer at once (at most 64 x 16): direct
                        CandCount base = 0;
                        if (lane == 0) base = atomicAdd(cand_count, (CandCount)tot);
                        base = __shfl(base, 0, 64);
                        int j = 0;
#pragma unroll
                        for (int r = 0; r < RT; r++)
#pragma unroll
                            for (int e = 0; e < 4; e++)
                                if ((pm >> (4 * r + e)) & 1u) {
                                    const int64_t idx = (int64_t)base + off + j++;
                                    if (idx < cand_cap) {
                                        Cand cd;
                                        cd.q = (int32_t)q;
                                        cd.pos = (int32_t)(row0 + 16 * r + 4 * rgrp + e);
                                        cd.val = (uint64_t)__float_as_uint(fmaf(-2.f, acc[r][e], qnn));
                                        cands[idx] = cd;
                                    }
                                }
                    } else {
                        int j = 0;
#pragma unroll
                        for (int r = 0; r < RT; r++)
#pragma unroll
                            for (int e = 0; e < 4; e++)
                                if ((pm >> (4 * r + e)) & 1u) {
                                    Cand cd;
                                    cd.q = (int32_t)q;
                                    cd.pos = (int32_t)(row0 + 16 * r + 4 * rgrp + e);
                                    cd.val = (uint64_t)__float_as_uint(fmaf(-2.f, acc[r][e], qnn));
                                    cbuf[nb + off + j++] = cd;
                                }
                        nb += tot;
                    }
                }
            }
            if (more) put(buf ^ 1);
            __syncthreads();
        }
    }
    if (nb) flush();
    if (lane == 0 && units) count_add(counters, CNT_TILE_PAIRS, (unsigned long long)units);
}

void slab_items(const SlabView &s, const uint64_t *leaf_mask, int ntiles, const SweepWork &w, hipStream_t st)
{
    fill_u32(w.counts, 3, 0u, st);   // pairs, items, work
    if (s.n_slabs == 0 || ntiles == 0) return;
    const unsigned grid = (unsigned)((s.n_slabs + kSlabsPerBlock - 1) / kSlabsPerBlock);
    hipLaunchKernelGGL(k_slab_items, dim3(grid), dim3(256), 0, st, s.leaf_lo, s.leaf_hi, s.n_slabs,
                       leaf_mask, ntiles, w.pair_tile, w.pair_mask, w.counts + 0, w.items, w.counts + 1);
    check_launch(__func__);
}

void mfma_sweep(const L2View &o, const SlabView &s, const QueryL2 &qv, const float *tqe, int64_t nq, int ntiles,
                const uint32_t *tomb, const SweepWork &w, Cand *cands, CandCount *cand_count, int64_t cand_cap,
                unsigned long long *counters, int grid_blocks, hipStream_t st)
{
    if (nq == 0 || s.n_slabs == 0) return;
    const float u = 5.9604645e-8f;  // 2^-24
    const int D = o.ksteps * 32;
    const float eps_a = 2.f * (D + 8) * u, eps_b = 2.f * (4 * D + 8) * u, eps_c = 8.f * u;
#define MS(KS)                                                                                                    \
    hipLaunchKernelGGL((k_mfma_sweep<KS, kRowTiles>), dim3((unsigned)grid_blocks), dim3(256), 0, st,                \
                       reinterpret_cast<const uint4 *>(o.X16t), o.xn, reinterpret_cast<const uint4 *>(qv.Q16t),   \
                       qv.qn, tqe, nq, s.emax, s.nmax, o.n, tomb, w.pair_tile, w.pair_mask, w.items, w.counts + 1, \
                       w.counts + 2, cands, cand_count, cand_cap, eps_a, eps_b, eps_c, counters)
    switch (o.ksteps) {
    case 1: MS(1); break;
    case 2: MS(2); break;
    case 3: MS(3); break;
    default: MS(4); break;
    }
#undef MS
    check_launch(__func__);
}

// ---------------------------------------------------------------------------
// Edit-distance object filtering over surviving (leaf, tile) pairs.  One wave
// per pair, lane = query.  Each object of the leaf is tested against every
// surviving query of the tile with the length bound | |q| - |o| | <= d(q,o)
// and Lemma 1 on every pivot (its row of the AoS pivot table is uniform
// across the wave); passing lanes are compacted with a ballot into a per-wave
// LDS buffer, which is flushed with one atomic reservation when full and at
// the end (one atomic per kObjBuf candidates instead of one per object).
// ---------------------------------------------------------------------------
constexpr int kObjBuf = 512;

template <int MP>
__global__ __launch_bounds__(256) void k_edit_objfilter(const int32_t *__restrict__ items,
                                                        const uint32_t *__restrict__ item_count, int64_t item_cap,
                                                        const uint64_t *__restrict__ leaf_mask, int ntiles,
                                                        const int32_t *__restrict__ leaf_first,
                                                        const int32_t *__restrict__ leaf_cnt,
                                                        const float *__restrict__ QP, const float *__restrict__ thr,
                                                        const int32_t *__restrict__ qlen, int64_t nq,
                                                        const uint8_t *__restrict__ PTa,
                                                        const int32_t *__restrict__ soff,
                                                        const uint32_t *__restrict__ tomb, Cand *__restrict__ cands,
                                                        CandCount *__restrict__ cand_count, int64_t cand_cap,
                                                        unsigned long long *__restrict__ counters)
{
    __shared__ int2 s_buf[4][kObjBuf];
    unsigned long long staged = 0, own = 0;   // wave-uniform work counts
    const int wave = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    int2 *buf = s_buf[wave];
    int nb = 0;   // buffered candidates (wave-uniform)
    auto flush = [&]() {
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        CandCount base = 0;
        if (lane == 0) base = atomicAdd(cand_count, (CandCount)nb);
        base = __shfl(base, 0, 64);
        for (int i = lane; i < nb; i += 64) {
            const int64_t idx = (int64_t)base + i;
            if (idx < cand_cap) {
                const int2 e = buf[i];
                Cand cd;
                cd.q = e.x;
                cd.pos = e.y;
                cd.val = 0;
                cands[idx] = cd;
            }
        }
        __builtin_amdgcn_wave_barrier();
        nb = 0;
    };
    int64_t nitems = *item_count;
    if (nitems > item_cap) nitems = item_cap;
    for (int64_t it = (int64_t)blockIdx.x * 4 + wave; it < nitems; it += (int64_t)gridDim.x * 4) {
        const int leaf = items[2 * it];
        const int tile = items[2 * it + 1];
        const uint64_t mask = leaf_mask[(size_t)leaf * ntiles + tile];
        if (mask == 0ull) continue;
        const int64_t q = (int64_t)tile * 64 + lane;
        const bool act = ((mask >> lane) & 1ull) && q < nq;
        staged += (unsigned long long)leaf_cnt[leaf];
        own += (unsigned long long)__popcll(dev::ballot(act)) * (unsigned long long)leaf_cnt[leaf];
        int qp[MP];
        int th = -1, ql = 0;
        if (act) {
#pragma unroll
            for (int i = 0; i < MP; i++) qp[i] = (int)QP[(size_t)q * MP + i];
            th = (int)thr[q];
            ql = qlen[q];
        } else {
#pragma unroll
            for (int i = 0; i < MP; i++) qp[i] = 0;
        }
        // the leaf's objects are staged 64 at a time, one per lane (length,
        // tombstone, pivot-table row), and broadcast to the tile's queries
        const int p0 = leaf_first[leaf];
        const int cnt = leaf_cnt[leaf];
        for (int b0 = 0; b0 < cnt; b0 += 64) {
            const int po = p0 + b0 + lane;
            const bool have = b0 + lane < cnt;
            int olen_l = 0;
            bool live_l = false;
            uint32_t rw[MP / 4];
            if (have) {
                live_l = !((tomb[po >> 5] >> (po & 31)) & 1u);
                olen_l = soff[po + 1] - soff[po];
                const uint32_t *r32 = reinterpret_cast<const uint32_t *>(PTa + (size_t)po * MP);
#pragma unroll
                for (int k2 = 0; k2 < MP / 4; k2++) rw[k2] = r32[k2];
            } else {
#pragma unroll
                for (int k2 = 0; k2 < MP / 4; k2++) rw[k2] = 0u;
            }
            // each lane (query) collects the staged objects it keeps, then
            // writes them contiguously: the candidate stream holds runs of
            // one query, which the grouping by query counts once per run
            uint64_t lv = dev::ballot(live_l), mine = 0ull;
            while (lv) {
                const int i = __ffsll((unsigned long long)lv) - 1;
                lv &= lv - 1ull;
                const int olen = __shfl(olen_l, i, 64);
                bool pass = act && abs(ql - olen) <= th;
#pragma unroll
                for (int k2 = 0; k2 < MP / 4; k2++) {
                    const uint32_t w = __shfl(rw[k2], i, 64);
#pragma unroll
                    for (int u = 0; u < 4; u++) pass = pass && abs(qp[4 * k2 + u] - (int)((w >> (8 * u)) & 0xffu)) <= th;
                }
                mine |= pass ? (1ull << i) : 0ull;
            }
            int total;
            const int before = dev::wave_excl_scan(__popcll(mine), &total);
            if (total == 0) continue;
            if (nb + total > kObjBuf) flush();
            if (total > kObjBuf) {   // more than the buffer holds: straight to memory
                CandCount base = 0;
                if (lane == 0) base = atomicAdd(cand_count, (CandCount)total);
                base = __shfl(base, 0, 64);
                int at = before;
                for (uint64_t m2 = mine; m2; m2 &= m2 - 1ull, at++) {
                    const int64_t idx = (int64_t)base + at;
                    if (idx < cand_cap) {
                        Cand cd;
                        cd.q = (int32_t)q;
                        cd.pos = p0 + b0 + (__ffsll((unsigned long long)m2) - 1);
                        cd.val = 0;
                        cands[idx] = cd;
                    }
                }
                continue;
            }
            int at = nb + before;
            for (uint64_t m2 = mine; m2; m2 &= m2 - 1ull, at++)
                buf[at] = make_int2((int)q, p0 + b0 + (__ffsll((unsigned long long)m2) - 1));
            nb += total;
        }
    }
    if (nb) flush();
    if (lane == 0 && staged) count_add(counters, CNT_FILTER_OBJS, staged);
    if (lane == 0 && own) count_add(counters, CNT_OWN_PAIRS, own);
}

void edit_objfilter(const TreeView &t, const int32_t *items, const uint32_t *item_count, int64_t item_cap,
                    const uint64_t *leaf_mask, int ntiles, const float *QP, const float *thr, const int32_t *qlen,
                    int64_t nq, const uint8_t *PTa, const int32_t *soff, const uint32_t *tomb, Cand *cands,
                    CandCount *cand_count, int64_t cand_cap, unsigned long long *counters, hipStream_t st)
{
    if (nq == 0) return;
    const unsigned blocks = 2048;
#define OF(MP)                                                                                                  \
    hipLaunchKernelGGL(k_edit_objfilter<MP>, dim3(blocks), dim3(256), 0, st, items, item_count, item_cap,        \
                       leaf_mask, ntiles, t.leaf_first, t.leaf_cnt, QP, thr, qlen, nq, PTa, soff, tomb, cands, \
                       cand_count, cand_cap, counters)
    if (t.mpad == 8) OF(8);
    else if (t.mpad == 16) OF(16);
    else OF(32);
#undef OF
    check_launch(__func__);
}

// ---------------------------------------------------------------------------
// Cache list (Sec. 4.4): brute force over every live cached object.
// ---------------------------------------------------------------------------
// Visibility of a cache slot to a query admitted at epoch e: inserted by an
// update of epoch e or earlier and not deleted by one of them.
__device__ __forceinline__ bool slot_visible(const uint32_t *cins, const uint32_t *cdel, int64_t s, uint32_t e)
{
    return cins[s] <= e && cdel[s] > e;
}

// L2: the cache scan is a dense (query x slot) distance tile, 64 queries x
// 64 slots per workgroup, each thread holding a 4 x 4 block of squared
// distances in registers.  The coordinates stream through LDS 32 at a time,
// stored dimension-major ([d][64 rows]) so that a thread reads its four
// query values (shared by the 16 threads of its row group: one broadcast)
// and its four slot values (consecutive across the 16 threads: no bank
// conflict) as float4.  Each pair accumulates (q_d - x_d)^2 in coordinate
// order (a float32 direct-difference sum, within (D + 1) 2^-24 relative of
// the exact distance; for L1 the sum of |q_d - x_d| in the same order);
// cut[q]: the emission cutoff (range radius, or for kNN the widened bound).
constexpr int kCacheTile = 64;
constexpr int kCacheChunk = 32;
template <bool L1>
__global__ __launch_bounds__(256) void k_cache_scan_l2(const float *__restrict__ Q32, int64_t nq, int dp,
                                                       const float *__restrict__ C32, CacheScan cs,
                                                       int64_t qtiles, const float *__restrict__ cut,
                                                       Cand *__restrict__ cands, CandCount *__restrict__ cand_count,
                                                       int64_t cand_cap, int angular)
{
    __shared__ float4 s_q[kCacheChunk][kCacheTile / 4];
    __shared__ float4 s_x[kCacheChunk][kCacheTile / 4];
    const int64_t st = blockIdx.x / qtiles, qt = blockIdx.x - st * qtiles;
    const int64_t s0 = st * kCacheTile, q0 = qt * kCacheTile;
    const int ns = (int)min<int64_t>(kCacheTile, cs.count - s0), nqt = (int)min<int64_t>(kCacheTile, nq - q0);
    const int tq = threadIdx.x >> 4, tx = threadIdx.x & 15;   // rows 4 tq.., 4 tx..
    float acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; i++)
#pragma unroll
        for (int j = 0; j < 4; j++) acc[i][j] = 0.f;
    float *sq = reinterpret_cast<float *>(s_q), *sx = reinterpret_cast<float *>(s_x);
    for (int d0 = 0; d0 < dp; d0 += kCacheChunk) {
        // 64 rows x 32 coordinates of each side, transposed into LDS
        for (int e = threadIdx.x; e < kCacheTile * kCacheChunk; e += blockDim.x) {
            const int r = e / kCacheChunk, c = e - r * kCacheChunk, d = d0 + c;
            sq[c * kCacheTile + r] = r < nqt && d < dp ? Q32[(size_t)(q0 + r) * dp + d] : 0.f;
            sx[c * kCacheTile + r] = r < ns && d < dp ? C32[(size_t)(s0 + r) * dp + d] : 0.f;
        }
        __syncthreads();
#pragma unroll 8
        for (int c = 0; c < kCacheChunk; c++) {
            const float4 qv = s_q[c][tq], xv = s_x[c][tx];
            const float qa[4] = {qv.x, qv.y, qv.z, qv.w}, xa[4] = {xv.x, xv.y, xv.z, xv.w};
#pragma unroll
            for (int i = 0; i < 4; i++)
#pragma unroll
                for (int j = 0; j < 4; j++) acc[i][j] = dev::dterm<L1>(acc[i][j], qa[i], xa[j]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 4; i++) {
        const int qi = 4 * tq + i;
        if (qi >= nqt) continue;
        const int64_t q = q0 + qi;
        const uint32_t e = cs.qep ? cs.qep[q] : cs.e_now;
        const float cq = cut[q];
#pragma unroll
        for (int j = 0; j < 4; j++) {
            const int sj = 4 * tx + j;
            if (sj >= ns) continue;
            const int64_t s = s0 + sj;
            const float d = dev::dfinish<L1>(acc[i][j]);
            if (d <= cq && slot_visible(cs.ins_ep, cs.del_ep, s, e)) {
                const CandCount idx = atomicAdd(cand_count, (CandCount)1);
                if ((int64_t)idx < cand_cap) {
                    Cand cd;
                    cd.q = (int32_t)q;
                    cd.pos = -1;
                    cd.val = ((uint64_t)__float_as_uint(dev::out_dist(d, angular != 0)) << 32) | cs.ids[s];
                    cands[idx] = cd;
                }
            }
        }
    }
}

void cache_scan_l2(const float *Q32, int64_t nq, int dp, const float *C32, const CacheScan &cs, const float *cut,
                   Cand *cands, CandCount *cand_count, int64_t cand_cap, bool angular, hipStream_t st, bool l1)
{
    if (nq == 0 || cs.count == 0) return;
    const int64_t stiles = (cs.count + kCacheTile - 1) / kCacheTile, qtiles = (nq + kCacheTile - 1) / kCacheTile;
    require(stiles * qtiles < ((int64_t)1 << 31), "cache_scan_l2: launch too large");
    if (l1)
        hipLaunchKernelGGL(k_cache_scan_l2<true>, dim3((unsigned)(stiles * qtiles)), dim3(256), 0, st, Q32, nq, dp,
                           C32, cs, qtiles, cut, cands, cand_count, cand_cap, 0);
    else
        hipLaunchKernelGGL(k_cache_scan_l2<false>, dim3((unsigned)(stiles * qtiles)), dim3(256), 0, st, Q32, nq, dp,
                           C32, cs, qtiles, cut, cands, cand_count, cand_cap, angular ? 1 : 0);
    check_launch(__func__);
}

// EDIT: one lane per (query, slot) pair, query as the pattern; length and
// pivot tests first (exact integers).
__global__ void k_cache_scan_edit(QueryEdit qv, EditView o, int64_t nq, const uint8_t *__restrict__ cchars, int cstride,
                                  const int32_t *__restrict__ clen, CacheScan cs, const float *__restrict__ base,
                                  Cand *__restrict__ cands, CandCount *__restrict__ cand_count, int64_t cand_cap)
{
    const int64_t pair = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (pair >= nq * cs.count) return;
    const int64_t q = pair / cs.count, c = pair % cs.count;
    if (!slot_visible(cs.ins_ep, cs.del_ep, c, cs.qep ? cs.qep[q] : cs.e_now)) return;
    const int cut = (int)floorf(fminf(base[q], 1e6f));
    const int plen = (int)(qv.off[q + 1] - qv.off[q]);
    const int tl = clen[c];
    if (abs(plen - tl) > cut) return;
    if (cs.cp) {
        const float *qp = cs.QP + (size_t)q * cs.mpad, *cp = cs.cp + (size_t)c * cs.mpad;
        for (int i = 0; i < cs.m; i++)
            if (fabsf(qp[i] - cp[i]) > (float)cut) return;
    }
    const int d = dev::myers_any(qv.peq + (size_t)q * o.rows * 4, plen, cchars + (size_t)c * cstride, tl, cut, o.lut);
    if (d <= cut) {
        const CandCount idx = atomicAdd(cand_count, (CandCount)1);
        if ((int64_t)idx < cand_cap) {
            Cand cd;
            cd.q = (int32_t)q;
            cd.pos = -1;
            cd.val = ((uint64_t)(uint32_t)d << 32) | cs.ids[c];
            cands[idx] = cd;
        }
    }
}

void cache_scan_edit(const QueryEdit &qv, const EditView &o, int64_t nq, const uint8_t *cchars, int cstride,
                     const int32_t *clen, const CacheScan &cs, const float *base, Cand *cands, CandCount *cand_count,
                     int64_t cand_cap, hipStream_t st)
{
    if (nq == 0 || cs.count == 0) return;
    const int64_t threads = nq * cs.count;
    require((threads + 255) / 256 < ((int64_t)1 << 31), "cache_scan_edit: launch too large");
    hipLaunchKernelGGL(k_cache_scan_edit, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, st, qv, o, nq,
                       cchars, cstride, clen, cs, base, cands, cand_count, cand_cap);
    check_launch(__func__);
}

}  // namespace k
}  // namespace gts
