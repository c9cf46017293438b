// Leaf-pivot kernels (edit distance): every leaf keeps its first object as a
// pivot p_L together with R_L = max over the leaf's objects o of d(o, p_L).
// By Lemma 1 with that pivot, d(q, o) >= d(q, p_L) - R_L for every o in L, so
// a leaf with d(q, p_L) > T_q + R_L holds no answer within T_q.  Distances are
// exact integers (bit-parallel Levenshtein), so the test needs no margin.
//
//   k_leaf_radius_edit : R_L at build time, one wave per leaf
//   k_edit_leaf_ball   : the leaf test for every (64-query tile, leaf) pair
//                        that survived the node filter; clears the mask bits
//                        of the queries it prunes
#include "dev_common.h"
#include "kernels.h"

namespace gts {
namespace k {

namespace {

// Match tables of a 64-query tile in LDS: word w of code c for the query of
// lane l sits at tab[(c * wt + w) * 64 + l] (conflict-free: every lane of a
// step reads the same code and word).
struct TilePeq {
    const uint64_t *tab;
    int wt;
    int lane;
    __device__ __forceinline__ uint64_t operator[](int i) const { return tab[((i >> 2) * wt + (i & 3)) * 64 + lane]; }
};

// Texts already mapped to codes.
struct NoLut {
    __device__ __forceinline__ int operator[](int c) const { return c; }
};

__device__ __forceinline__ int wave_max_i(int v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
    return v;
}

}  // namespace

// ---------------------------------------------------------------------------
// R_L: one wave per leaf; the pivot (the leaf's first object) is the Myers
// pattern, its match table per wave in LDS; lanes stride over the objects.
// Empty leaves get R_L = -inf (their test never passes).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_leaf_radius_edit(EditView o, const int32_t *__restrict__ leaf_first,
                                                          const int32_t *__restrict__ leaf_cnt, int64_t n_leaves,
                                                          float *__restrict__ leafR)
{
    __shared__ uint64_t s_tab[4][257 * 4];
    __shared__ uint8_t s_lut[256];
    const int wave = dev::uniform((int)(threadIdx.x >> 6)), lane = dev::lane_id();
    const int64_t leaf = (int64_t)blockIdx.x * 4 + wave;
    uint64_t *tab = s_tab[wave];
    for (int i = lane; i < o.rows * 4; i += 64) tab[i] = 0ull;
    for (int i = threadIdx.x; i < 256; i += blockDim.x) s_lut[i] = o.lut[i];
    __syncthreads();
    int cnt = 0, p0 = 0, plen = 0;
    if (leaf < n_leaves) {
        cnt = leaf_cnt[leaf];
        p0 = leaf_first[leaf];
        if (cnt > 0) {
            const int32_t s0 = o.soff[p0];
            plen = o.soff[p0 + 1] - s0;
            for (int b = lane; b < plen; b += 64) {
                const int c = s_lut[o.chars[s0 + b]];
                if (c < o.rows - 1)
                    atomicOr(reinterpret_cast<unsigned long long *>(&tab[c * 4 + (b >> 6)]),
                             (unsigned long long)(1ull << (b & 63)));
            }
        }
    }
    __syncthreads();
    if (leaf >= n_leaves) return;
    int r = 0;
    for (int j = lane; j < cnt; j += 64) {
        const int32_t s0 = o.soff[p0 + j];
        const int tl = o.soff[p0 + j + 1] - s0;
        r = max(r, dev::myers_any(tab, plen, o.chars + s0, tl, 1 << 30, s_lut));
    }
    r = wave_max_i(r);
    if (lane == 0) leafR[leaf] = cnt > 0 ? (float)r : -INFINITY;
}

void leaf_radius_edit(const EditView &o, const int32_t *leaf_first, const int32_t *leaf_cnt, int64_t n_leaves,
                      float *leafR, hipStream_t st)
{
    if (n_leaves == 0) return;
    hipLaunchKernelGGL(k_leaf_radius_edit, dim3((unsigned)((n_leaves + 3) / 4)), dim3(256), 0, st, o, leaf_first,
                       leaf_cnt, n_leaves, leafR);
    check_launch(__func__);
}

// ---------------------------------------------------------------------------
// Leaf test.  Workgroup = (tile, chunk of kLeafChunk leaves), four waves; the
// 64 lanes of a wave are the tile's 64 queries (each the Myers pattern of its
// own lane) and a wave walks its leaves one at a time: the pivot string is the
// common text, staged as codes in LDS.  Per lane the cutoff is T_q + R_L, with
// the early exit of the bit-parallel recurrence; the length difference alone
// prunes first.  The tile's match tables sit in LDS when they fit (TAB), else
// lanes read their own query's table from global memory.
// ---------------------------------------------------------------------------
constexpr int kLeafChunk = 256;
constexpr int kTileTabWords = 4096;   // 32 KiB of LDS

struct GlobalPeq {
    const uint64_t *tab;
    __device__ __forceinline__ uint64_t operator[](int i) const { return tab[i]; }
};

template <int W, bool TAB>
__global__ __launch_bounds__(256) void k_edit_leaf_ball(EditView o, QueryEdit qv, const int32_t *__restrict__ qlen,
                                                        const int32_t *__restrict__ leaf_first,
                                                        const float *__restrict__ leafR, int64_t n_leaves,
                                                        const float *__restrict__ T, int64_t nq, int ntiles,
                                                        uint64_t *__restrict__ leaf_mask)
{
    extern __shared__ uint64_t s_tab[];   // rows * W * 64 words when TAB
    __shared__ uint8_t s_code[4][256];
    __shared__ uint8_t s_lut[256];
    const int wave = dev::uniform((int)(threadIdx.x >> 6)), lane = dev::lane_id();
    const int tile = (int)(blockIdx.x % ntiles);
    const int64_t chunk = blockIdx.x / ntiles;
    const int64_t q = (int64_t)tile * 64 + lane;
    const bool qok = q < nq;
    for (int i = threadIdx.x; i < 256; i += blockDim.x) s_lut[i] = o.lut[i];
    if (TAB) {
        // s_tab[(c * W + w) * 64 + j] = word w of code c of query tile*64 + j
        const int words = o.rows * W * 64;
        for (int i = threadIdx.x; i < words; i += blockDim.x) {
            const int j = i & 63, w = (i >> 6) % W, c = (i >> 6) / W;
            const int64_t qq = (int64_t)tile * 64 + j;
            s_tab[i] = qq < nq ? qv.peq[((size_t)qq * o.rows + c) * 4 + w] : 0ull;
        }
    }
    __syncthreads();
    const int plen = qok ? qlen[q] : 0;
    const int tq = qok ? (int)T[q] : -1;
    const uint64_t *gtab = qv.peq + (size_t)(qok ? q : 0) * o.rows * 4;
    for (int64_t li = wave; li < kLeafChunk; li += 4) {
        const int64_t leaf = chunk * kLeafChunk + li;
        if (leaf >= n_leaves) break;
        uint64_t *slot = leaf_mask + (size_t)leaf * ntiles + tile;
        const uint64_t m = *slot;
        if (m == 0ull) continue;
        const float R = leafR[leaf];
        if (R < 0.f) {
            if (lane == 0) *slot = 0ull;
            continue;
        }
        const int32_t pf = leaf_first[leaf];
        const int32_t s0 = o.soff[pf];
        const int tl = o.soff[pf + 1] - s0;
        for (int b = lane; b < tl; b += 64) s_code[wave][b] = s_lut[o.chars[s0 + b]];
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const int cut = tq + (int)R;
        bool pass = ((m >> lane) & 1ull) && abs(plen - tl) <= cut;
        if (pass) {
            int d;
            if (TAB) d = dev::myers_distance<W>(TilePeq{s_tab, W, lane}, plen, s_code[wave], tl, cut, NoLut{});
            else d = dev::myers_distance<W>(GlobalPeq{gtab}, plen, s_code[wave], tl, cut, NoLut{});
            pass = d <= cut;
        }
        const uint64_t nm = dev::ballot(pass);
        if (lane == 0) *slot = nm;
        __builtin_amdgcn_wave_barrier();
    }
}

void edit_leaf_ball(const EditView &o, const QueryEdit &qv, const int32_t *qlen, const int32_t *leaf_first,
                    const float *leafR, int64_t n_leaves, const float *T, int64_t nq, int ntiles, int max_qlen,
                    uint64_t *leaf_mask, hipStream_t st)
{
    if (nq == 0 || n_leaves == 0) return;
    const int W = std::max(1, (max_qlen + 63) / 64);
    const int64_t chunks = (n_leaves + kLeafChunk - 1) / kLeafChunk;
    const unsigned grid = (unsigned)(chunks * ntiles);
    const bool tab = (int64_t)o.rows * W * 64 <= kTileTabWords;
    const size_t shm = tab ? (size_t)o.rows * W * 64 * sizeof(uint64_t) : 0;
#define EB(WW, TB)                                                                                                  \
    hipLaunchKernelGGL((k_edit_leaf_ball<WW, TB>), dim3(grid), dim3(256), shm, st, o, qv, qlen, leaf_first, leafR, \
                       n_leaves, T, nq, ntiles, leaf_mask)
#define EBW(TB)             \
    switch (W) {            \
    case 1: EB(1, TB); break; \
    case 2: EB(2, TB); break; \
    case 3: EB(3, TB); break; \
    default: EB(4, TB); break; \
    }
    if (tab) EBW(true) else EBW(false)
#undef EBW
#undef EB
    check_launch(__func__);
}

}  // namespace k
}  // namespace gts
