// Float32 candidate selection for L2 (precision GTS_FP32): Lemma 1 on the
// pivot table for every object of the surviving (leaf, query tile) pairs.
//
//   k_mask_items   : the (leaf, tile) pairs whose leaf mask keeps some query,
//                    compacted leaf-major (consecutive items share a leaf, so
//                    its pivot-table columns are read from L2 after the first)
//   k_l2_objfilter : one wave per item, lane = query of the tile.  The leaf's
//                    objects are staged 64 at a time: lane j reads object j's
//                    column of the SoA table PT[p][o] (one coalesced 256-byte
//                    read per pivot) into an LDS row, and every lane then
//                    reads each staged row as a broadcast (same address on
//                    all lanes) and applies Lemma 1 -- o can be an answer of
//                    q only if |d(q, p) - d(o, p)| <= thr[q] for every pivot p,
//                    thr carrying the float32 error margin of both
//                    distances.  Kept objects leave as candidates without an
//                    estimate (every one gets a float32 distance).
#include "dev_common.h"
#include "gts_internal.h"
#include "kernels.h"

namespace gts {
namespace k {

__global__ __launch_bounds__(256) void k_mask_items(const uint64_t *__restrict__ leaf_mask, int64_t n_leaves,
                                                    int ntiles, int32_t *__restrict__ items,
                                                    uint32_t *__restrict__ item_count, int64_t item_cap)
{
    const int64_t total = n_leaves * ntiles;
    const int lane = threadIdx.x & 63;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t b0 = (int64_t)blockIdx.x * blockDim.x + (threadIdx.x & ~63u); b0 < total; b0 += stride) {
        const int64_t i = b0 + lane;
        const bool pass = i < total && leaf_mask[i] != 0ull;
        const uint64_t m = dev::ballot(pass);
        if (!m) continue;
        uint32_t base = 0;
        if (lane == 0) base = atomicAdd(item_count, (uint32_t)__popcll(m));
        base = __shfl(base, 0, 64);
        const int64_t at = (int64_t)base + dev::lanes_below(m);
        if (pass && at < item_cap) {
            items[2 * at] = (int32_t)(i / ntiles);
            items[2 * at + 1] = (int32_t)(i % ntiles);
        }
    }
}

void mask_items(const uint64_t *leaf_mask, int64_t n_leaves, int ntiles, int32_t *items, uint32_t *item_count,
                int64_t item_cap, hipStream_t st)
{
    const int64_t total = n_leaves * ntiles;
    if (total == 0) return;
    const unsigned grid = (unsigned)std::min<int64_t>((total + 255) / 256, 4096);
    hipLaunchKernelGGL(k_mask_items, dim3(grid), dim3(256), 0, st, leaf_mask, n_leaves, ntiles, items, item_count,
                       item_cap);
    check_launch(__func__);
}

constexpr int kObjBuf32 = 512;

template <int MP>
__global__ __launch_bounds__(256) void k_l2_objfilter(const int32_t *__restrict__ items,
                                                      const uint32_t *__restrict__ item_count, int64_t item_cap,
                                                      const uint64_t *__restrict__ leaf_mask, int ntiles,
                                                      const int32_t *__restrict__ leaf_first,
                                                      const int32_t *__restrict__ leaf_cnt,
                                                      const float *__restrict__ QP, const float *__restrict__ thr,
                                                      int64_t nq, const float *__restrict__ PT, int64_t n,
                                                      const uint32_t *__restrict__ tomb, Cand *__restrict__ cands,
                                                      CandCount *__restrict__ cand_count, int64_t cand_cap,
                                                      unsigned long long *__restrict__ counters)
{
    unsigned long long staged = 0;   // objects staged (wave-uniform)
    constexpr int RS = MP + 4;   // LDS row stride in floats (16-byte rows, banks spread)
    __shared__ float4 s_rows[4][64 * RS / 4];
    __shared__ int2 s_buf[4][kObjBuf32];
    const int wave = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    float *rows = reinterpret_cast<float *>(s_rows[wave]);
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
        const int64_t q = (int64_t)tile * 64 + lane;
        const bool act = ((mask >> lane) & 1ull) && q < nq;
        float qp[MP];
        float th = -INFINITY;
#pragma unroll
        for (int i = 0; i < MP; i++) qp[i] = act ? QP[(size_t)q * MP + i] : 0.f;
        if (act) th = thr[q];
        const int p0 = leaf_first[leaf];
        const int cnt = leaf_cnt[leaf];
        staged += (unsigned long long)cnt;
        for (int b0 = 0; b0 < cnt; b0 += 64) {
            const int64_t po = (int64_t)p0 + b0 + lane;
            const bool have = b0 + lane < cnt;
            const bool live_l = have && !((tomb[po >> 5] >> (po & 31)) & 1u);
            __builtin_amdgcn_wave_barrier();
#pragma unroll
            for (int p = 0; p < MP; p++) rows[lane * RS + p] = have ? PT[(size_t)p * n + po] : 0.f;
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            // each lane (query) collects the staged objects it keeps, then
            // writes them contiguously (runs of one query for the grouping)
            uint64_t lv = dev::ballot(live_l), mine = 0ull;
            while (lv) {
                const int i = __ffsll((unsigned long long)lv) - 1;
                lv &= lv - 1ull;
                const float4 *r4 = reinterpret_cast<const float4 *>(rows + i * RS);
                float g = 0.f;
#pragma unroll
                for (int p4 = 0; p4 < MP / 4; p4++) {
                    const float4 v = r4[p4];
                    g = fmaxf(g, fabsf(qp[4 * p4 + 0] - v.x));
                    g = fmaxf(g, fabsf(qp[4 * p4 + 1] - v.y));
                    g = fmaxf(g, fabsf(qp[4 * p4 + 2] - v.z));
                    g = fmaxf(g, fabsf(qp[4 * p4 + 3] - v.w));
                }
                mine |= (act && g <= th) ? (1ull << i) : 0ull;
            }
            int total;
            const int before = dev::wave_excl_scan(__popcll(mine), &total);
            if (total == 0) continue;
            if (nb + total > kObjBuf32) flush();
            if (total > kObjBuf32) {   // more than the buffer holds: straight to memory
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
}

void l2_objfilter(const TreeView &t, const int32_t *items, const uint32_t *item_count, int64_t item_cap,
                  const uint64_t *leaf_mask, int ntiles, const float *QP, const float *thr, int64_t nq, const float *PT,
                  int64_t n, const uint32_t *tomb, Cand *cands, CandCount *cand_count, int64_t cand_cap,
                  unsigned long long *counters, hipStream_t st)
{
    if (nq == 0) return;
    const unsigned blocks = 2048;
#define OF(MP)                                                                                                  \
    hipLaunchKernelGGL(k_l2_objfilter<MP>, dim3(blocks), dim3(256), 0, st, items, item_count, item_cap,          \
                       leaf_mask, ntiles, t.leaf_first, t.leaf_cnt, QP, thr, nq, PT, n, tomb, cands, cand_count, \
                       cand_cap, counters)
    if (t.mpad == 8) OF(8);
    else if (t.mpad == 16) OF(16);
    else OF(32);
#undef OF
    check_launch(__func__);
}

}  // namespace k
}  // namespace gts
