// Leaf-pivot kernels (L2): every leaf keeps one of its own objects as a
// pivot p_L together with R_L = max over the leaf's objects o of d(o, p_L).
// By Lemma 1 with that pivot, every o in L has d(q, o) >= d(q, p_L) - R_L, so
// a leaf with d(q, p_L) - R_L > T holds no answer within T.  The distances
// d(q, p_L) for all (query, leaf) pairs come from the same bf16 MFMA tiles as
// the object distances, with a rigorous error margin.
//
//   k_leaf_near : the NB leaves whose pivots are nearest to each query (by the
//                 bf16 estimate; a heuristic choice -- only used to pick
//                 which exact distances bound the kNN radius and how queries
//                 are grouped into tiles)
//   k_leaf_ball : the leaf test above for every (64-query tile, leaf),
//                 ANDed into the node filter's leaf masks
//   k_bound_near: kNN radius bound: the k-th smallest exact float32 distance
//                 over the objects of the nearest leaves
#include "dev_common.h"
#include "kernels.h"

namespace gts {
namespace k {

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float floatx4_t __attribute__((ext_vector_type(4)));

__device__ __forceinline__ bf16x8_t frag(uint4 v)
{
    bf16x8_t r;
    __builtin_memcpy(&r, &v, sizeof(r));
    return r;
}

// ---------------------------------------------------------------------------
// Nearest leaf pivots.  One workgroup per 16-query block (the MFMA B operand,
// in registers); its four waves split the leaf pivots, which stream through
// as A fragments, 16 per MFMA row block, the next block's fragments loading
// while the current one is multiplied.  Each lane keeps a sorted top-NB of
// its estimates (insertion by selects, no branches per slot); the 16 lists
// holding one query (4 lanes x 4 waves) merge through LDS.
// ---------------------------------------------------------------------------
template <int KS, int NB>
__global__ __launch_bounds__(256) void k_leaf_near(const uint4 *__restrict__ PL16t, const float *__restrict__ pln,
                                                   int64_t lpad, const uint4 *__restrict__ Q16t, int64_t nq,
                                                   int32_t *__restrict__ near)
{
    __shared__ float s_d[4][64][NB];
    __shared__ int32_t s_l[4][64][NB];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t blk = blockIdx.x;                        // 16-query block
    float bd[NB];
    int32_t bl[NB];
#pragma unroll
    for (int i = 0; i < NB; i++) {
        bd[i] = INFINITY;
        bl[i] = -1;
    }
    uint4 B[KS];
#pragma unroll
    for (int s = 0; s < KS; s++) B[s] = Q16t[(blk * KS + s) * 64 + lane];
    const int rg = lane >> 4;
    const int64_t G = lpad / 16;
    uint4 A[KS];
    if (wave < G) {
#pragma unroll
        for (int s = 0; s < KS; s++) A[s] = PL16t[((int64_t)wave * KS + s) * 64 + lane];
    }
    for (int64_t g = wave; g < G; g += 4) {
        uint4 An[KS];
        const int64_t gn = g + 4 < G ? g + 4 : g;
#pragma unroll
        for (int s = 0; s < KS; s++) An[s] = PL16t[(gn * KS + s) * 64 + lane];
        float pv[4];
#pragma unroll
        for (int e = 0; e < 4; e++) pv[e] = pln[16 * g + 4 * rg + e];
        floatx4_t acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int s = 0; s < KS; s++)
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(frag(A[s]), frag(B[s]), acc, 0, 0, 0);
#pragma unroll
        for (int e = 0; e < 4; e++) {
            const int32_t leaf = (int32_t)(16 * g + 4 * rg + e);
            const float v = fmaf(-2.f, acc[e], pv[e]);   // d^2 - ||q||^2
            if (v < bd[NB - 1]) {
                float cv = v;
                int32_t cl = leaf;
#pragma unroll
                for (int i = 0; i < NB; i++) {
                    const bool lt = cv < bd[i];
                    const float td = lt ? bd[i] : cv;
                    const int32_t tl = lt ? bl[i] : cl;
                    bd[i] = lt ? cv : bd[i];
                    bl[i] = lt ? cl : bl[i];
                    cv = td;
                    cl = tl;
                }
            }
        }
#pragma unroll
        for (int s = 0; s < KS; s++) A[s] = An[s];
    }
#pragma unroll
    for (int i = 0; i < NB; i++) {
        s_d[wave][lane][i] = bd[i];
        s_l[wave][lane][i] = bl[i];
    }
    __syncthreads();
    if (wave != 0 || lane >= 16) return;
    const int64_t q = blk * 16 + lane;
    if (q >= nq) return;
    // merge the 16 lists of this query: list j = (wave j >> 2, lane lane + 16 (j & 3))
    int idx[16];
#pragma unroll
    for (int j = 0; j < 16; j++) idx[j] = 0;
    for (int i = 0; i < NB; i++) {
        int best = -1;
        float bv = INFINITY;
#pragma unroll
        for (int j = 0; j < 16; j++) {
            if (idx[j] < NB) {
                const float v = s_d[j >> 2][lane + 16 * (j & 3)][idx[j]];
                if (best < 0 || v < bv) {
                    bv = v;
                    best = j;
                }
            }
        }
        int32_t leaf = -1;
#pragma unroll
        for (int j = 0; j < 16; j++)
            if (j == best) {
                leaf = s_l[j >> 2][lane + 16 * (j & 3)][idx[j]];
                idx[j]++;
            }
        near[q * NB + i] = leaf;
    }
}

void leaf_near(const uint16_t *PL16t, const float *pln, int64_t lpad, int ksteps, const uint16_t *Q16t, int64_t nq,
               int32_t *near, hipStream_t st)
{
    if (nq == 0) return;
    require(ksteps >= 1 && ksteps <= 4, "leaf_near: rows wider than 128 floats");
    const unsigned grid = (unsigned)((nq + 15) / 16);
#define LN(KS)                                                                                              \
    hipLaunchKernelGGL((k_leaf_near<KS, kNearLeaves>), dim3(grid), dim3(256), 0, st,                        \
                       reinterpret_cast<const uint4 *>(PL16t), pln, lpad, reinterpret_cast<const uint4 *>(Q16t), \
                       nq, near)
    switch (ksteps) {
    case 1: LN(1); break;
    case 2: LN(2); break;
    case 3: LN(3); break;
    default: LN(4); break;
    }
#undef LN
    check_launch(__func__);
}

// ---------------------------------------------------------------------------
// Leaf ball test.  One wave per (64-query tile, 64-leaf group): 4 leaf row
// blocks x 4 query column blocks of MFMA.  A (query, leaf) pair passes when
// the lower bound of d(q, p_L) minus R_L does not exceed T_q; per leaf the 64
// pass bits of the tile are assembled through LDS and ANDed into the mask.
// ---------------------------------------------------------------------------
template <int KS>
__global__ __launch_bounds__(256) void k_leaf_ball(const uint4 *__restrict__ PL16t, const float *__restrict__ pln,
                                                   const float *__restrict__ ple, const float *__restrict__ leafR,
                                                   int64_t n_leaves, int64_t ngroups, const uint4 *__restrict__ Q16t,
                                                   const float *__restrict__ qn, const float *__restrict__ qe,
                                                   const float *__restrict__ T, int64_t nq, int ntiles,
                                                   uint64_t *__restrict__ leaf_mask, float eps_a, float eps_b,
                                                   const int32_t *__restrict__ leaf_cnt,
                                                   unsigned long long *__restrict__ counters)
{
    __shared__ uint16_t s_bits[4][64][4];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t w0 = (int64_t)blockIdx.x * 4 + wave;
    const bool live = w0 < (int64_t)ntiles * ngroups;   // no early exit: the block meets a barrier below
    const int64_t w = live ? w0 : 0;
    const int tile = (int)(w / ngroups);
    const int64_t lg = w % ngroups;
    const int rg = lane >> 4, col = lane & 15;
    // the box test's verdicts for this tile: only 16-query blocks with a
    // surviving (query, leaf) pair in this leaf group are tested again
    const int64_t my_leaf = lg * 64 + lane;
    const uint64_t box_m = live && my_leaf < n_leaves ? leaf_mask[(size_t)my_leaf * ntiles + tile] : 0ull;
    uint64_t box_any = 0;                                 // bit c: some leaf keeps a query of block c
#pragma unroll
    for (int c = 0; c < 4; c++) box_any |= dev::ballot(((box_m >> (16 * c)) & 0xffffull) != 0) ? (1ull << c) : 0ull;
    uint4 A[4][KS];
    float pn[4][4], pe[4][4], R[4][4];
#pragma unroll
    for (int r = 0; r < 4; r++) {
#pragma unroll
        for (int s = 0; s < KS; s++)
            A[r][s] = box_any ? PL16t[((lg * 4 + r) * KS + s) * 64 + lane] : make_uint4(0, 0, 0, 0);
#pragma unroll
        for (int e = 0; e < 4; e++) {
            const int64_t leaf = lg * 64 + 16 * r + 4 * rg + e;
            pn[r][e] = pln[leaf];
            pe[r][e] = ple[leaf];
            R[r][e] = leaf < n_leaves ? leafR[leaf] : -INFINITY;
        }
    }
    // the query blocks' fragments and parameters, all requested before the
    // first is used (blocks whose pairs all failed the box test skip theirs)
    uint4 Ball[4][KS];
    float qnv[4], qev[4], tqv[4];
#pragma unroll
    for (int c = 0; c < 4; c++) {
        const bool use = (box_any >> c) & 1ull;
        const int64_t q = (int64_t)tile * 64 + 16 * c + col;
#pragma unroll
        for (int s = 0; s < KS; s++)
            Ball[c][s] = use ? Q16t[(((int64_t)tile * 4 + c) * KS + s) * 64 + lane] : make_uint4(0, 0, 0, 0);
        const bool qv = use && q < nq;
        qnv[c] = qv ? qn[q] : 0.f;
        qev[c] = qv ? qe[q] : 0.f;
        tqv[c] = qv ? T[q] : -INFINITY;
    }
#pragma unroll
    for (int c = 0; c < 4; c++) {
        if (!((box_any >> c) & 1ull)) {
            // every pair of this block already failed the box test
#pragma unroll
            for (int e = 0; e < 4; e++)
                if (col == 0)
#pragma unroll
                    for (int r = 0; r < 4; r++) s_bits[wave][16 * r + 4 * rg + e][c] = 0;
            continue;
        }
        const int64_t q = (int64_t)tile * 64 + 16 * c + col;
        const uint4 *B = Ball[c];
        const float qnn = qnv[c], qerr = qev[c], tq = tqv[c];
        floatx4_t acc[4];
#pragma unroll
        for (int r = 0; r < 4; r++) acc[r] = floatx4_t{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int s = 0; s < KS; s++)
#pragma unroll
            for (int r = 0; r < 4; r++)
                acc[r] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(frag(A[r][s]), frag(B[s]), acc[r], 0, 0, 0);
#pragma unroll
        for (int r = 0; r < 4; r++)
#pragma unroll
            for (int e = 0; e < 4; e++) {
                const float d2 = qnn + fmaf(-2.f, acc[r][e], pn[r][e]);
                const float eps = eps_a * (qnn + pn[r][e]) + eps_b * sqrtf(qnn * pn[r][e]) + 8.f * 5.9604645e-8f * fabsf(d2);
                const float lo = sqrtf(fmaxf(d2 - eps, 0.f)) - qerr - pe[r][e];
                const bool pass = q < nq && lo - R[r][e] <= tq;
                const uint64_t b = dev::ballot(pass);
                // lanes 16j..16j+15 hold leaf 16r + 4j + e, queries 0..15
                if (col == 0) s_bits[wave][16 * r + 4 * rg + e][c] = (uint16_t)(b >> (16 * rg));
            }
    }
    __syncthreads();
    unsigned long long own = 0;   // (query, object) pairs of the surviving (query, leaf) pairs
    if (live && my_leaf < n_leaves && box_m) {
        const uint64_t m = (uint64_t)s_bits[wave][lane][0] | ((uint64_t)s_bits[wave][lane][1] << 16) |
                           ((uint64_t)s_bits[wave][lane][2] << 32) | ((uint64_t)s_bits[wave][lane][3] << 48);
        leaf_mask[(size_t)my_leaf * ntiles + tile] = box_m & m;
        own = (unsigned long long)__popcll(box_m & m) * (unsigned long long)leaf_cnt[my_leaf];
    }
    for (int o2 = 32; o2 > 0; o2 >>= 1) own += __shfl_xor(own, o2, 64);
    if (lane == 0 && own) count_add(counters, CNT_OWN_PAIRS, own);
}

void leaf_ball(const uint16_t *PL16t, const float *pln, const float *ple, const float *leafR, int64_t n_leaves,
               int ksteps, const uint16_t *Q16t, const float *qn, const float *qe, const float *T, int64_t nq,
               int ntiles, uint64_t *leaf_mask, const int32_t *leaf_cnt, unsigned long long *counters,
               hipStream_t st)
{
    if (nq == 0 || n_leaves == 0) return;
    require(ksteps >= 1 && ksteps <= 4, "leaf_ball: rows wider than 128 floats");
    const int64_t ngroups = (n_leaves + 63) / 64;
    const int64_t waves = (int64_t)ntiles * ngroups;
    const unsigned grid = (unsigned)((waves + 3) / 4);
    const float u = 5.9604645e-8f;
    const int D = ksteps * 32;
    const float eps_a = 2.f * (D + 8) * u, eps_b = 2.f * (4 * D + 8) * u;
#define LB(KS)                                                                                                 \
    hipLaunchKernelGGL(k_leaf_ball<KS>, dim3(grid), dim3(256), 0, st, reinterpret_cast<const uint4 *>(PL16t), pln, \
                       ple, leafR, n_leaves, ngroups, reinterpret_cast<const uint4 *>(Q16t), qn, qe, T, nq, ntiles, \
                       leaf_mask, eps_a, eps_b, leaf_cnt, counters)
    switch (ksteps) {
    case 1: LB(1); break;
    case 2: LB(2); break;
    case 3: LB(3); break;
    default: LB(4); break;
    }
#undef LB
    check_launch(__func__);
}

// ---------------------------------------------------------------------------
// kNN radius bound from the nearest leaves: exact float32 distances to the
// objects of the query's nearest leaves (in order, while at most kWinObj
// objects and until at least max(k, target) were taken); the k-th smallest
// live distance bounds the k-th nearest neighbour distance from above.
//
// One workgroup per query.  The queries arrive sorted by home leaf, so
// neighbouring queries read the same leaves: runs of consecutive queries go
// to the same XCD (workgroups are dealt to the 8 XCDs round robin), where the
// second read of a leaf hits that XCD's L2, and the runs are dealt to the
// XCDs in turn so each gets its share of every part of the query order.  The window plan is one wave-wide scan;
// object rows and tombstone words of kBoundUnroll objects per 16-lane group
// are loaded before any of them is used.
// ---------------------------------------------------------------------------
constexpr int kWinObj = 2048;
constexpr int kBoundUnroll = 4;
constexpr int64_t kBoundRun = 64;   // consecutive queries per run dealt to one XCD

__global__ __launch_bounds__(256) void k_bound_near(const int32_t *__restrict__ near,
                                                    const int32_t *__restrict__ leaf_first,
                                                    const int32_t *__restrict__ leaf_cnt, const float *__restrict__ X32,
                                                    int dp, const float *__restrict__ Q32,
                                                    const int32_t *__restrict__ kq, int64_t nq,
                                                    const uint32_t *__restrict__ tomb, int target,
                                                    float *__restrict__ tq, unsigned long long *__restrict__ counters,
                                                    int only_unbounded)
{
    __shared__ float s_d[kWinObj];
    __shared__ int s_first[kNearLeaves], s_start[kNearLeaves + 1];
    __shared__ int s_nl;
    // runs of kBoundRun consecutive queries are dealt to the XCDs in turn
    // (gridDim.x is a multiple of 8 kBoundRun)
    const int64_t i = blockIdx.x >> 3, run = (i / kBoundRun) * 8 + (blockIdx.x & 7);
    const int64_t q = run * kBoundRun + i % kBoundRun;
    if (q >= nq) return;
    const int k = kq[q];
    if (k <= 0) return;
    if (only_unbounded && tq[q] < INFINITY) return;   // bounded by the MFMA kernel
    // the window: a prefix of the nearest leaves; each condition that ends it
    // (a missing leaf, more than kWinObj objects, max(k, target) reached) is
    // monotone along the list, so lane i is in the window iff it passes all
    if (threadIdx.x < 64) {
        const int i = (int)threadIdx.x;
        const int32_t leaf = i < kNearLeaves ? near[q * kNearLeaves + i] : -1;
        const int cnt = leaf >= 0 ? leaf_cnt[leaf] : 0;
        const int first = leaf >= 0 ? leaf_first[leaf] : 0;
        int total;
        const int excl = dev::wave_excl_scan(cnt, &total);
        const uint64_t missing = dev::ballot(leaf < 0);
        const int want = k > target ? k : target;
        const bool in = (missing & ((2ull << i) - 1ull)) == 0 && excl + cnt <= kWinObj && excl < want;
        const uint64_t inm = dev::ballot(in);
        if (in) {
            s_first[i] = first;
            s_start[i + 1] = excl + cnt;
        }
        if (i == 0) {
            s_start[0] = 0;
            s_nl = __popcll(inm);
        }
    }
    __syncthreads();
    const int nl = s_nl, count = s_start[nl];
    if (threadIdx.x == 0) count_add(counters, CNT_BOUND_EVALS, (unsigned long long)count);
    if (count < k) {
        if (threadIdx.x == 0) tq[q] = INFINITY;
        return;
    }
    // 16 lanes per object, strided coordinates, query slice in registers
    const int sl = threadIdx.x & 15, grp = (int)(threadIdx.x >> 4);
    float qr[8];
#pragma unroll
    for (int t = 0; t < 8; t++) qr[t] = sl + 16 * t < dp ? Q32[(size_t)q * dp + sl + 16 * t] : 0.f;
    for (int j0 = 0; j0 < count; j0 += 16 * kBoundUnroll) {
        float xv[kBoundUnroll][8];
        uint32_t tw[kBoundUnroll];
        int pos[kBoundUnroll];
#pragma unroll
        for (int u = 0; u < kBoundUnroll; u++) {
            const int j = j0 + 16 * u + grp;
            int p = 0;
            if (j < count) {
                int e = 0;
                while (e + 1 < nl && s_start[e + 1] <= j) e++;
                p = s_first[e] + (j - s_start[e]);
            }
            pos[u] = p;
            const float *x = X32 + (size_t)p * dp;
#pragma unroll
            for (int t = 0; t < 8; t++) xv[u][t] = j < count && sl + 16 * t < dp ? x[sl + 16 * t] : 0.f;
            tw[u] = j < count ? tomb[p >> 5] : 0u;
        }
#pragma unroll
        for (int u = 0; u < kBoundUnroll; u++) {
            const int j = j0 + 16 * u + grp;
            // coordinates beyond dp are zero on both sides: fmaf(0, 0, acc) == acc
            float acc = 0.f;
#pragma unroll
            for (int t = 0; t < 8; t++) {
                const float df = qr[t] - xv[u][t];
                acc = fmaf(df, df, acc);
            }
#pragma unroll
            for (int o = 8; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 16);
            const bool dead = (tw[u] >> (pos[u] & 31)) & 1u;
            if (j < count && sl == 0) s_d[j] = dead ? INFINITY : sqrtf(acc);
        }
    }
    const int P = dev::next_pow2(count);
    for (int j = count + threadIdx.x; j < P; j += blockDim.x) s_d[j] = INFINITY;
    dev::bitonic_sort(s_d, P);
    if (threadIdx.x == 0) tq[q] = s_d[k - 1];
}

void bound_near(const int32_t *near, const int32_t *leaf_first, const int32_t *leaf_cnt, const float *X32, int dp,
                const float *Q32, const int32_t *kq, int64_t nq, const uint32_t *tomb, int target, float *tq,
                unsigned long long *counters, hipStream_t st, bool only_unbounded)
{
    if (nq == 0) return;
    require(dp <= 128, "bound_near: rows wider than 128 floats");
    const unsigned grid = (unsigned)((nq + 8 * kBoundRun - 1) / (8 * kBoundRun) * (8 * kBoundRun));
    hipLaunchKernelGGL(k_bound_near, dim3(grid), dim3(256), 0, st, near, leaf_first, leaf_cnt, X32, dp, Q32,
                       kq, nq, tomb, target, tq, counters, only_unbounded ? 1 : 0);
    check_launch(__func__);
}

// ---------------------------------------------------------------------------
// kNN radius bound by bf16 MFMA.  One workgroup per 16-query block of the
// home order.  The block's window is a set of distinct whole 16-row groups of
// the leaf order: the groups covering the leaves of its kNN queries'
// nearest-leaf lists, list position by list position (every query's nearest
// leaf first), at most kMbGroups of them.  Every kNN query of the block whose
// nearest leaf lies wholly in the window gets
// the bf16 estimate of its squared distance to every live object of the
// window (its own nearest leaves and its neighbours'), turned into the upper
// end of the estimate's proven interval (the same bound as the candidate
// selection); the k-th smallest upper end is at least the k-th smallest true
// distance over the window, whose objects are live objects of the index, so
// it bounds the k-th nearest neighbour distance from above.  A query whose
// exact-kernel window (the leading leaves of its list) is not wholly in the
// block's window gets +inf and the exact kernel takes it (its k-th value
// would otherwise come from the leaves of other queries of the block, which
// can be far from it).  The window's group list: per list entry its leaf's group
// range, kept at the leaf's first occurrence (a scan gives each kept range
// its place), then each group kept at its first occurrence (neighbouring
// leaves share their boundary group; an object counted twice would make the
// k-th value too small).
// ---------------------------------------------------------------------------
constexpr int kMbGroups = 64;                 // 16-row groups per window
constexpr int kMbRows = 16 * kMbGroups;
constexpr int kMbEntries = 16 * kNearLeaves;  // (list position, query) entries of a block
constexpr int kMbWaves = 8;                   // waves per workgroup
constexpr int kMbBatch = 2;                   // groups whose loads a wave issues together
static_assert(kMbGroups % (kMbWaves * kMbBatch) == 0, "whole batches of groups");
static_assert(kMbEntries == 128, "two waves hold the entries");

template <int KS>
__global__ __launch_bounds__(64 * kMbWaves) void k_bound_mfma(const uint4 *__restrict__ X16t, const float *__restrict__ xn,
                                                    const float *__restrict__ xe, int64_t n,
                                                    const int32_t *__restrict__ near,
                                                    const int32_t *__restrict__ leaf_first,
                                                    const int32_t *__restrict__ leaf_cnt,
                                                    const uint4 *__restrict__ Q16t, const float *__restrict__ qn,
                                                    const float *__restrict__ qe, const int32_t *__restrict__ kq,
                                                    int64_t nq, const uint32_t *__restrict__ tomb, int target,
                                                    float eps_a,
                                                    float eps_b, float eps_c, float *__restrict__ tq,
                                                    unsigned long long *__restrict__ counters)
{
    __shared__ int32_t s_leaf[kMbEntries], s_glo[kMbEntries], s_first[kMbEntries];
    __shared__ int32_t s_rlo[kMbEntries], s_rend[kMbEntries];   // the entry leaf's rows
    __shared__ uint8_t s_full[kMbEntries];
    __shared__ int32_t s_grp[kMbGroups];
    __shared__ int s_tot[2];
    __shared__ float s_hi[16][kMbRows + 1];
    const int64_t blk = blockIdx.x;
    const int t = (int)threadIdx.x, wave = t >> 6, lane = t & 63;
    // entry t = (list position t / 16, query t % 16): its leaf's group range
    int gn = 0;
    if (t < kMbEntries) {
        const int j = t >> 4, c = t & 15;
        const int64_t q = blk * 16 + c;
        int32_t leaf = -1;
        int glo = 0, first = 0, cnt = 0;
        if (q < nq && kq[q] > 0) {
            leaf = near[q * kNearLeaves + j];
            cnt = leaf >= 0 ? leaf_cnt[leaf] : 0;
            if (cnt > 0) {
                first = leaf_first[leaf];
                glo = first >> 4;
                gn = ((first + cnt - 1) >> 4) - glo + 1;
            } else {
                leaf = -1;
                cnt = 0;
            }
        }
        s_leaf[t] = leaf;
        s_glo[t] = glo;
        s_rlo[t] = q < nq && kq[q] > 0 && near[q * kNearLeaves + j] >= 0 ? first : -1;   // -1: the list ended
        s_rend[t] = first + cnt;
    }
    __syncthreads();
    int off = 0;
    if (t < kMbEntries) {
        const int32_t leaf = s_leaf[t];
        int fst = t;                           // the first entry holding this leaf
        for (int i = t - 1; i >= 0 && leaf >= 0; i--)
            if (s_leaf[i] == leaf) fst = i;
        if (fst != t) gn = 0;
        s_first[t] = fst;
        int tot;
        off = dev::wave_excl_scan(gn, &tot);
        if (lane == 0) s_tot[wave] = tot;
    }
    __syncthreads();
    const int total = s_tot[0] + s_tot[1];
    if (total == 0) {
        // no leaf in any list of the block (uniform): its kNN queries, if
        // any, go to the exact kernel
        if (t < 16 && blk * 16 + t < nq && kq[blk * 16 + t] > 0) tq[blk * 16 + t] = INFINITY;
        return;
    }
    if (t < kMbEntries) {
        if (wave == 1) off += s_tot[0];
        const int glo = s_glo[t];
        for (int u = 0; u < gn && off + u < kMbGroups; u++) s_grp[off + u] = glo + u;
        // a leaf's groups are all in the window when its first entry's
        // range ended inside it
        s_full[t] = s_leaf[t] >= 0 && gn > 0 && off + gn <= kMbGroups ? 1 : 0;
    }
    const int ng = total < kMbGroups ? total : kMbGroups;
    __syncthreads();
    int32_t my_grp = -1;
    if (t < ng) {
        my_grp = s_grp[t];
        for (int i = 0; i < t; i++)
            if (s_grp[i] == my_grp) my_grp = -1;
    }
    __syncthreads();
    if (t < kMbGroups) s_grp[t] = t < ng ? my_grp : -1;
    __syncthreads();
    // estimates: wave w takes groups w, w + 8, ...; the loads of
    // kMbBatch groups are issued before any of them is used.  Lane
    // (rgrp, col) holds rows 4 rgrp + e of a group for query col.
    const int col = lane & 15, rgrp = lane >> 4;
    const int64_t qc = blk * 16 + col;
    uint4 B[KS];
#pragma unroll
    for (int s2 = 0; s2 < KS; s2++) B[s2] = Q16t[(blk * KS + s2) * 64 + lane];
    const float qnn = qn[qc], qerr = qe[qc];   // (the query arrays are padded to whole 64-query tiles)
    for (int gb = wave; gb < kMbGroups; gb += kMbWaves * kMbBatch) {
        uint4 A[kMbBatch][KS];
        float xnv[kMbBatch][4], xev[kMbBatch][4];
        uint32_t lv[kMbBatch];                 // live bits of the lane's 4 rows
#pragma unroll
        for (int bb = 0; bb < kMbBatch; bb++) {
            const int32_t g = s_grp[gb + bb * kMbWaves];
            lv[bb] = 0u;
#pragma unroll
            for (int s2 = 0; s2 < KS; s2++)
                A[bb][s2] = g >= 0 ? X16t[((int64_t)g * KS + s2) * 64 + lane] : make_uint4(0, 0, 0, 0);
#pragma unroll
            for (int e = 0; e < 4; e++) {
                const int64_t row = (int64_t)(g >= 0 ? g : 0) * 16 + 4 * rgrp + e;
                xnv[bb][e] = g >= 0 ? xn[row] : 0.f;
                xev[bb][e] = g >= 0 ? xe[row] : 0.f;
                if (g >= 0 && row < n && !((tomb[row >> 5] >> (row & 31)) & 1u)) lv[bb] |= 1u << e;
            }
        }
#pragma unroll
        for (int bb = 0; bb < kMbBatch; bb++) {
            floatx4_t acc = {-0.5f * xnv[bb][0], -0.5f * xnv[bb][1], -0.5f * xnv[bb][2], -0.5f * xnv[bb][3]};
#pragma unroll
            for (int s2 = 0; s2 < KS; s2++)
                acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(frag(A[bb][s2]), frag(B[s2]), acc, 0, 0, 0);
            const int gi = gb + bb * kMbWaves;
#pragma unroll
            for (int e = 0; e < 4; e++) {
                const float est = fmaf(-2.f, acc[e], qnn);
                const float eps = eps_a * (qnn + xnv[bb][e]) + eps_b * sqrtf(qnn * xnv[bb][e]) + eps_c * fabsf(est);
                const float hi = sqrtf(fmaxf(est + eps, 0.f)) + qerr + xev[bb][e];
                s_hi[col][gi * 16 + 4 * rgrp + e] = (lv[bb] >> e) & 1u ? hi : INFINITY;
            }
        }
    }
    __syncthreads();
    // per query the k-th smallest upper end: wave w takes queries 2w and
    // 2w + 1, each lane kMbRows / 64 values; the smallest v with
    // #{hi <= v} >= k by a binary search over the float bits (hi >= 0: float
    // order = bit order)
    unsigned long long evals = 0;
    for (int cq = 0; cq < 16 / kMbWaves; cq++) {
        const int c = (16 / kMbWaves) * wave + cq;
        const int64_t q = blk * 16 + c;
        const int k = q < nq ? kq[q] : 0;     // (uniform over the wave)
        if (k <= 0) continue;
        // a query whose nearest leaf is not wholly in the window has no
        // good bound here: the exact kernel takes it
        const int32_t l0 = s_leaf[c];          // entry (position 0, query c)
        if (l0 < 0 || !s_full[s_first[c]]) {
            if (lane == 0) tq[q] = INFINITY;
            continue;
        }
        // the exact kernel's window for this query (the prefix of its list
        // up to max(k, target) objects, at most kWinObj) must lie wholly in
        // the block's window, which then holds a superset of its objects:
        // the k-th value is no looser than the exact kernel's but for the
        // bf16 interval.  Otherwise (the k-th value would come from other
        // queries' leaves, which can be far away) the exact kernel takes it.
        const int want = k > target ? k : target;
        int acc = 0;
        bool inside = true;
        for (int j = 0; j < kNearLeaves && acc < want; j++) {
            const int e = j * 16 + c;
            if (s_rlo[e] < 0) break;
            const int cnt = s_rend[e] - s_rlo[e];
            if (acc + cnt > kWinObj) break;
            if (cnt > 0 && !s_full[s_first[e]]) {
                inside = false;
                break;
            }
            acc += cnt;
        }
        if (!inside) {
            if (lane == 0) tq[q] = INFINITY;
            continue;
        }
        uint32_t hvb[kMbRows / 64];
        int live = 0;
#pragma unroll
        for (int u = 0; u < kMbRows / 64; u++) {
            hvb[u] = __float_as_uint(s_hi[c][lane + 64 * u]);
            live += __popcll(dev::ballot(hvb[u] < 0x7f800000u));
        }
        float b = INFINITY;
        if (k <= live) {
            uint32_t lo_v = 0u, hi_v = 0x7f800000u;
            while (lo_v < hi_v) {
                const uint32_t mid = lo_v + ((hi_v - lo_v) >> 1);
                int cnt = 0;
#pragma unroll
                for (int u = 0; u < kMbRows / 64; u++) cnt += __popcll(dev::ballot(hvb[u] <= mid));
                if (cnt >= k) hi_v = mid;
                else lo_v = mid + 1u;
            }
            b = __uint_as_float(lo_v);
        }
        if (lane == 0) tq[q] = b;
        evals += (unsigned long long)live;
    }
    if (lane == 0 && evals) count_add(counters, CNT_BOUND_EVALS, evals);
}

void bound_mfma(const uint16_t *X16t, const float *xn, const float *xe, int64_t n, int ksteps, const int32_t *near,
                const int32_t *leaf_first, const int32_t *leaf_cnt, const uint16_t *Q16t, const float *qn,
                const float *qe, const int32_t *kq, int64_t nq, const uint32_t *tomb, int target, float *tq,
                unsigned long long *counters, hipStream_t st)
{
    if (nq == 0) return;
    require(ksteps >= 1 && ksteps <= 4, "bound_mfma: rows wider than 128 floats");
    const float u = 5.9604645e-8f;
    const int D = ksteps * 32;
    const float eps_a = 2.f * (D + 8) * u, eps_b = 2.f * (4 * D + 8) * u, eps_c = 8.f * u;
    const unsigned grid = (unsigned)((nq + 15) / 16);
#define BM(KS)                                                                                                 \
    hipLaunchKernelGGL(k_bound_mfma<KS>, dim3(grid), dim3(64 * kMbWaves), 0, st,                                \
                       reinterpret_cast<const uint4 *>(X16t), xn,                                                \
                       xe, n, near, leaf_first, leaf_cnt, reinterpret_cast<const uint4 *>(Q16t), qn, qe, kq, nq,   \
                       tomb, target, eps_a, eps_b, eps_c, tq, counters)
    switch (ksteps) {
    case 1: BM(1); break;
    case 2: BM(2); break;
    case 3: BM(3); break;
    default: BM(4); break;
    }
#undef BM
    check_launch(__func__);
}

// ---------------------------------------------------------------------------
// Query permutation helpers.
// ---------------------------------------------------------------------------
__global__ void k_gather_rows(const float *__restrict__ src, const int32_t *__restrict__ perm, int64_t rows, int dp,
                              float *__restrict__ dst)
{
    const int64_t i = (int64_t)blockIdx.x;
    if (i >= rows) return;
    const float *s = src + (size_t)perm[i] * dp;
    float *d = dst + (size_t)i * dp;
    for (int c = threadIdx.x; c < dp; c += blockDim.x) d[c] = s[c];
}

void gather_rows(const float *src, const int32_t *perm, int64_t rows, int dp, float *dst, hipStream_t st)
{
    if (rows == 0) return;
    hipLaunchKernelGGL(k_gather_rows, dim3((unsigned)rows), dim3(64), 0, st, src, perm, rows, dp, dst);
    check_launch(__func__);
}

__global__ void k_gather_i32(const int32_t *__restrict__ src, const int32_t *__restrict__ perm, int64_t rows, int width,
                             int32_t *__restrict__ dst)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= rows * width) return;
    const int64_t r = i / width, c = i % width;
    dst[i] = src[(size_t)perm[r] * width + c];
}

void gather_i32(const int32_t *src, const int32_t *perm, int64_t rows, int width, int32_t *dst, hipStream_t st)
{
    if (rows == 0) return;
    const int64_t n = rows * width;
    hipLaunchKernelGGL(k_gather_i32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, src, perm, rows, width, dst);
    check_launch(__func__);
}

__global__ void k_permute_queries(const int32_t *__restrict__ perm, int64_t nq, const float *__restrict__ base_s,
                                  float *__restrict__ base_d, const int32_t *__restrict__ kq_s,
                                  int32_t *__restrict__ kq_d, const float *__restrict__ qp_s, float *__restrict__ qp_d,
                                  int mpad, const float *__restrict__ q32_s, float *__restrict__ q32_d, int dp,
                                  const int32_t *__restrict__ near_s, int32_t *__restrict__ near_d, int nnear)
{
    const int64_t i = blockIdx.x;
    if (i >= nq) return;
    const int64_t p = perm[i];
    if (threadIdx.x == 0) {
        base_d[i] = base_s[p];
        kq_d[i] = kq_s[p];
    }
    for (int c = threadIdx.x; c < mpad; c += blockDim.x) qp_d[i * mpad + c] = qp_s[p * mpad + c];
    if (q32_s)
        for (int c = threadIdx.x; c < dp; c += blockDim.x) q32_d[i * dp + c] = q32_s[p * dp + c];
    if (near_s)
        for (int c = threadIdx.x; c < nnear; c += blockDim.x) near_d[i * nnear + c] = near_s[p * nnear + c];
}

void permute_queries(const int32_t *perm, int64_t nq, const float *base_s, float *base_d, const int32_t *kq_s,
                     int32_t *kq_d, const float *qp_s, float *qp_d, int mpad, const float *q32_s, float *q32_d,
                     int dp, const int32_t *near_s, int32_t *near_d, int nnear, hipStream_t st)
{
    if (nq == 0) return;
    hipLaunchKernelGGL(k_permute_queries, dim3((unsigned)nq), dim3(64), 0, st, perm, nq, base_s, base_d, kq_s, kq_d,
                       qp_s, qp_d, mpad, q32_s, q32_d, dp, near_s, near_d, nnear);
    check_launch(__func__);
}

// Strings: dst string i <- src string perm[i] (dst offsets precomputed).
__global__ void k_gather_strings(const uint8_t *__restrict__ src, const int64_t *__restrict__ src_off,
                                 const int32_t *__restrict__ perm, int64_t n, const int64_t *__restrict__ dst_off,
                                 uint8_t *__restrict__ dst)
{
    const int64_t i = blockIdx.x;
    if (i >= n) return;
    const int64_t a = src_off[perm[i]], len = src_off[perm[i] + 1] - a, b = dst_off[i];
    for (int64_t j = threadIdx.x; j < len; j += blockDim.x) dst[b + j] = src[a + j];
}

void gather_strings(const uint8_t *src, const int64_t *src_off, const int32_t *perm, int64_t n, const int64_t *dst_off,
                    uint8_t *dst, hipStream_t st)
{
    if (n == 0) return;
    hipLaunchKernelGGL(k_gather_strings, dim3((unsigned)n), dim3(64), 0, st, src, src_off, perm, n, dst_off, dst);
    check_launch(__func__);
}

// Answers computed in permuted query order -> original order:
// dst segment of original query perm[i] <- src segment i.
__global__ void k_unpermute(const int64_t *__restrict__ src_off, const int64_t *__restrict__ dst_off,
                            const int32_t *__restrict__ perm, int64_t nq, const int64_t *__restrict__ src_ids,
                            const uint32_t *__restrict__ src_dist, int64_t *__restrict__ dst_ids,
                            uint32_t *__restrict__ dst_dist)
{
    const int64_t i = blockIdx.x;
    if (i >= nq) return;
    const int64_t a = src_off[i], n = src_off[i + 1] - a;
    const int64_t b = dst_off[perm[i]];
    for (int64_t j = threadIdx.x; j < n; j += blockDim.x) {
        dst_ids[b + j] = src_ids[a + j];
        dst_dist[b + j] = src_dist[a + j];
    }
}

void unpermute(const int64_t *src_off, const int64_t *dst_off, const int32_t *perm, int64_t nq, const int64_t *src_ids,
               const uint32_t *src_dist, int64_t *dst_ids, uint32_t *dst_dist, hipStream_t st)
{
    if (nq == 0) return;
    hipLaunchKernelGGL(k_unpermute, dim3((unsigned)nq), dim3(64), 0, st, src_off, dst_off, perm, nq, src_ids, src_dist,
                       dst_ids, dst_dist);
    check_launch(__func__);
}

}  // namespace k
}  // namespace gts
