// Leaf-pivot kernels (edit distance): every leaf keeps its first object as a
// pivot p_L together with R_L = max over the leaf's objects o of d(o, p_L).
// By Lemma 1 with that pivot, d(q, o) >= d(q, p_L) - R_L for every o in L, so
// a leaf with d(q, p_L) > T_q + R_L holds no answer within T_q.  Distances are
// exact integers (bit-parallel Levenshtein), so the test needs no margin.
//
//   k_leaf_radius_edit : R_L at build time, one wave per leaf
//   k_edit_cell_test   : the cell test for every (64-query tile, cell)
//   k_edit_leaf_query  : the leaf test for every (query, leaf of a cell that
//                        passed for it); writes the leaf masks and the list
//                        of (leaf, tile) pairs that object filtering walks
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
// Cell test.  Workgroup = (64-query tile, 256 cells), one cell per lane: the
// lane keeps its cell's box, length range and radius in registers and walks
// the tile's queries, whose pivot distances, lengths, thresholds and pivot
// centres sit in LDS (every lane reads the same entry: a broadcast).  A cell
// passes the cheap tests for a query when its box over the global pivot
// distances (Lemma 1 on every pivot), its string-length range and Lemma 1
// with the query's pivot centre admit T_q; those (query, cell) pairs then take
// the exact ball test d(q, centre) <= T_q + R_c in the lane that holds the
// cell, the query's match table in LDS when the tile's tables fit (TAB), the
// centre string as the text.
// ---------------------------------------------------------------------------
constexpr int kTileTabWords = 4096;   // 32 KiB of LDS

struct GlobalPeq {
    const uint64_t *tab;
    __device__ __forceinline__ uint64_t operator[](int i) const { return tab[i]; }
};

// The tile's match tables into LDS: s_tab[(c * W + w) * 64 + j] = word w of
// code c of the tile's query j (zero for positions past nq); position p of
// the tile order holds query order[p] (order may be null: the identity).
template <int W>
__device__ __forceinline__ void load_tile_tab(uint64_t *s_tab, const QueryEdit &qv, int rows, int tile, int64_t nq,
                                              const int32_t *__restrict__ order)
{
    const int words = rows * W * 64;
    for (int i = threadIdx.x; i < words; i += blockDim.x) {
        const int j = i & 63, w = (i >> 6) % W, c = (i >> 6) / W;
        const int64_t qq = (int64_t)tile * 64 + j;
        const int64_t qi = qq < nq ? (order ? order[qq] : qq) : 0;
        s_tab[i] = qq < nq ? qv.peq[((size_t)qi * rows + c) * 4 + w] : 0ull;
    }
}

template <int W, int MP, bool TAB>
__global__ __launch_bounds__(256) void k_edit_cell_test(EditView o, QueryEdit qv, const int32_t *__restrict__ qlen,
                                                        const float *__restrict__ QP, const float *__restrict__ T,
                                                        int64_t nq, int ntiles, CellView cv,
                                                        const int32_t *__restrict__ piv,
                                                        const int32_t *__restrict__ pivd,
                                                        int32_t *__restrict__ qcells, int32_t *__restrict__ qcnt,
                                                        unsigned long long *__restrict__ counters,
                                                        const int32_t *__restrict__ order)
{
    extern __shared__ uint64_t s_tab[];
    __shared__ float s_qp[64][MP];
    __shared__ int s_q[64], s_plen[64], s_tq[64], s_hc[64], s_hd[64];
    __shared__ uint8_t s_lut[256];
    const int tile = (int)(blockIdx.x % ntiles);
    const int64_t chunk = blockIdx.x / ntiles;
    const int nj = (int)min((int64_t)64, nq - (int64_t)tile * 64);
    for (int j = threadIdx.x; j < 64; j += blockDim.x) {
        const int64_t p = (int64_t)tile * 64 + j;
        const bool ok = j < nj;
        const int64_t q = ok ? (order ? order[p] : p) : 0;
        const int h = ok && piv ? piv[q] : -1;
        s_q[j] = (int)q;
        s_plen[j] = ok ? qlen[q] : 0;
        s_tq[j] = ok ? (int)T[q] : -1;
        s_hc[j] = h;
        s_hd[j] = h >= 0 ? pivd[q] : 0;
    }
    for (int i = threadIdx.x; i < 64 * MP; i += blockDim.x) {
        const int j = i / MP;
        const int64_t p = (int64_t)tile * 64 + j;
        s_qp[j][i % MP] = j < nj ? QP[(size_t)(order ? order[p] : p) * MP + i % MP] : 0.f;
    }
    for (int i = threadIdx.x; i < 256; i += blockDim.x) s_lut[i] = o.lut[i];
    if (TAB) load_tile_tab<W>(s_tab, qv, o.rows, tile, nq, order);
    __syncthreads();
    const int64_t c = chunk * 256 + threadIdx.x;
    const float R = c < cv.n ? cv.R[c] : -INFINITY;
    long long tests = c < cv.n ? nj : 0;
    uint64_t m = 0ull;   // bit j: query j passed the cheap tests
    if (R >= 0.f) {
        float lo[MP], hi[MP];
        const float *b = cv.box + (size_t)c * 2 * MP;
#pragma unroll
        for (int i = 0; i < MP; i++) {
            lo[i] = b[i];
            hi[i] = b[MP + i];
        }
        const int lmin = cv.len[2 * c], lmax = cv.len[2 * c + 1], ri = (int)R;
#pragma unroll 16
        for (int j = 0; j < nj; j++) {
            const int tq = s_tq[j], pl = s_plen[j], h = s_hc[j];
            float g = -INFINITY;
#pragma unroll
            for (int i = 0; i < MP; i++) g = fmaxf(g, fmaxf(lo[i] - s_qp[j][i], s_qp[j][i] - hi[i]));
            bool pass = g <= (float)tq && lmin - pl <= tq && pl - lmax <= tq;
            if (h >= 0) pass = pass && abs((int)cv.dist[(size_t)h * cv.n + c] - s_hd[j]) <= tq + ri;
            m |= pass ? (1ull << j) : 0ull;
        }
        if (m) {
            const int32_t s0 = cv.off[c];
            const int tl = cv.off[c + 1] - s0;
            const uint8_t *text = cv.chars + s0;
            while (m) {
                const int j = __ffsll((unsigned long long)m) - 1;
                m &= m - 1ull;
                const int pl = s_plen[j], cut = s_tq[j] + ri, wq = (pl + 63) >> 6;
                int d;
                if (cut <= 63) {
                    if (TAB) d = dev::myers_banded(TilePeq{s_tab, W, j}, W, pl, text, tl, cut, s_lut);
                    else d = dev::myers_banded(GlobalPeq{qv.peq + (size_t)s_q[j] * o.rows * 4}, 4, pl, text, tl, cut,
                                               s_lut);
                } else if (TAB) {
                    const TilePeq t{s_tab, W, j};
                    if (W >= 2 && wq <= 1) d = dev::myers_distance<1>(t, pl, text, tl, cut, s_lut);
                    else if (W >= 3 && wq <= 2) d = dev::myers_distance<2>(t, pl, text, tl, cut, s_lut);
                    else if (W >= 4 && wq <= 3) d = dev::myers_distance<3>(t, pl, text, tl, cut, s_lut);
                    else d = dev::myers_distance<W>(t, pl, text, tl, cut, s_lut);
                } else {
                    const GlobalPeq t{qv.peq + (size_t)s_q[j] * o.rows * 4};
                    if (W >= 2 && wq <= 1) d = dev::myers_distance<1>(t, pl, text, tl, cut, s_lut);
                    else if (W >= 3 && wq <= 2) d = dev::myers_distance<2>(t, pl, text, tl, cut, s_lut);
                    else if (W >= 4 && wq <= 3) d = dev::myers_distance<3>(t, pl, text, tl, cut, s_lut);
                    else d = dev::myers_distance<W>(t, pl, text, tl, cut, s_lut);
                }
                if (d <= cut) {
                    const int64_t p = (int64_t)tile * 64 + j;
                    const int slot = atomicAdd(&qcnt[p], 1);
                    if (slot < kQueryCells) qcells[(size_t)p * kQueryCells + slot] = (int32_t)c;
                }
            }
        }
    }
    for (int o2 = 32; o2 > 0; o2 >>= 1) tests += __shfl_xor(tests, o2, 64);
    if (dev::lane_id() == 0 && tests) count_add(counters, CNT_NODE_TESTS, (unsigned long long)tests);
}

// Leaves are reached from the cells that passed, query by query: one wave per
// query (its match table in LDS).  The (cell, leaf) pairs of the query's list
// are numbered across the cells (a wave prefix sum of their leaf counts in
// LDS) and dealt to the lanes 64 at a time, each lane scanning its leaf pivot
// as the text with the cutoff T_q + R_L.  A leaf that spans several cells is
// tested from the first of them on the list.  A query whose list overflowed
// takes every leaf once.  A
// passing (query, leaf) pair sets the query's bit in leaf_mask[leaf][tile];
// the first bit set in a word appends (leaf, tile) to the item list
// (leaf_mask starts zeroed).
template <int W>
__global__ __launch_bounds__(256) void k_edit_leaf_query(EditView o, QueryEdit qv, const int32_t *__restrict__ qlen,
                                                         const float *__restrict__ T,
                                                         const int32_t *__restrict__ leaf_first,
                                                         const float *__restrict__ leafR,
                                                         const int32_t *__restrict__ leaf_cell,
                                                         const int32_t *__restrict__ cell_leaf, int64_t n_cells,
                                                         int64_t n_leaves, const int32_t *__restrict__ qcells,
                                                         const int32_t *__restrict__ qcnt, int64_t nq, int ntiles,
                                                         unsigned long long *__restrict__ leaf_mask,
                                                         int32_t *__restrict__ items, uint32_t *__restrict__ item_count,
                                                         int64_t item_cap)
{
    extern __shared__ uint64_t s_tabs[];   // 4 x rows x 4 words
    __shared__ uint8_t s_lut[256];
    __shared__ int32_t s_cells[4][kQueryCells];
    __shared__ int32_t s_pre[4][kQueryCells + 1];   // leaf pairs before each listed cell
    const int wave = dev::uniform((int)(threadIdx.x >> 6)), lane = dev::lane_id();
    const int64_t q = (int64_t)blockIdx.x * 4 + wave;
    const bool qok = q < nq;
    uint64_t *tab = s_tabs + (size_t)wave * o.rows * 4;
    for (int i = threadIdx.x; i < 256; i += blockDim.x) s_lut[i] = o.lut[i];
    int cnt = 0;
    if (qok) {
        for (int i = lane; i < o.rows * 4; i += 64) tab[i] = qv.peq[(size_t)q * o.rows * 4 + i];
        cnt = qcnt[q];
        for (int i = lane; i < min(cnt, kQueryCells); i += 64) s_cells[wave][i] = qcells[(size_t)q * kQueryCells + i];
    }
    __syncthreads();
    if (!qok || cnt == 0) return;
    const bool all = cnt > kQueryCells;   // the list overflowed: every leaf
    const int plen = qlen[q];
    const int wq = (plen + 63) >> 6;
    const int tq = (int)T[q];
    const int tile = (int)(q >> 6);
    const unsigned long long bit = 1ull << (q & 63);
    int total;
    if (all) {
        total = (int)n_leaves;
    } else {
        int nl = 0;
        if (lane < cnt) {
            const int c = s_cells[wave][lane];
            nl = max(0, cell_leaf[2 * c + 1] - cell_leaf[2 * c] + 1);
        }
        const int ex = dev::wave_excl_scan(nl, &total);
        if (lane < cnt) s_pre[wave][lane] = ex;
        if (lane == 0) s_pre[wave][cnt] = total;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    auto listed = [&](int e) {
        bool f = false;
        for (int i = 0; i < cnt; i++) f = f || s_cells[wave][i] == e;
        return f;
    };
    for (int i0 = 0; i0 < total; i0 += 64) {
        const int i = i0 + lane;
        bool ok = i < total;
        int leaf = 0;
        if (ok) {
            if (all) {
                leaf = i;
            } else {
                int lo = 0, hi = cnt - 1;   // the listed cell whose pair range holds i
                while (lo < hi) {
                    const int mid = (lo + hi + 1) >> 1;
                    if (s_pre[wave][mid] <= i) lo = mid;
                    else hi = mid - 1;
                }
                const int c = s_cells[wave][lo];
                leaf = cell_leaf[2 * c] + (i - s_pre[wave][lo]);
                for (int e = leaf_cell[2 * leaf]; e < c; e++) ok = ok && !listed(e);
            }
        }
        {
            const float R = ok ? leafR[leaf] : -1.f;
            ok = ok && R >= 0.f;
            if (ok) {
                const int32_t s0 = o.soff[leaf_first[leaf]];
                const int tl = o.soff[leaf_first[leaf] + 1] - s0;
                const int cut = tq + (int)R;
                if (abs(plen - tl) > cut) {
                    ok = false;
                } else {
                    int d;
                    if (cut <= 63) d = dev::myers_banded(tab, 4, plen, o.chars + s0, tl, cut, s_lut);
                    else if (W >= 2 && wq <= 1) d = dev::myers_distance<1>(tab, plen, o.chars + s0, tl, cut, s_lut);
                    else if (W >= 3 && wq <= 2) d = dev::myers_distance<2>(tab, plen, o.chars + s0, tl, cut, s_lut);
                    else if (W >= 4 && wq <= 3) d = dev::myers_distance<3>(tab, plen, o.chars + s0, tl, cut, s_lut);
                    else d = dev::myers_distance<W>(tab, plen, o.chars + s0, tl, cut, s_lut);
                    ok = d <= cut;
                }
            }
            if (ok) {
                const unsigned long long old = atomicOr(leaf_mask + (size_t)leaf * ntiles + tile, bit);
                if (old == 0ull) {
                    const uint32_t idx = atomicAdd(item_count, 1u);
                    if (idx < item_cap) {
                        items[2 * (size_t)idx] = leaf;
                        items[2 * (size_t)idx + 1] = tile;
                    }
                }
            }
        }
    }
}

// Pivot centre per query: one wave per query.  Lanes stride over the query's
// q-grams and add one vote to every centre listed in the q-gram's bucket
// (16-bit LDS counters, two per word, one row of n_cells per wave; a query
// has fewer than 2^16 q-grams); the four centres with the most votes (ties:
// lower rank) get their distance, one lane each, exact up to 63 (banded
// recurrence), and the nearest of them is the pivot.  No vote at all (a
// query shorter than a q-gram, or sharing none) or no centre within 63: no
// pivot.
__global__ __launch_bounds__(256) void k_edit_pivot(EditView o, QueryEdit qv, int64_t nq, CellView cv,
                                                    int32_t *__restrict__ piv, int32_t *__restrict__ pivd)
{
    // LDS: per wave nw vote words (nw even), then per wave the query's match
    // table (rows x 4 words), which the four distances read per character
    extern __shared__ uint32_t s_votes[];
    __shared__ uint8_t s_lut[256];
    const int wave = dev::uniform((int)(threadIdx.x >> 6)), lane = dev::lane_id();
    const int64_t q = (int64_t)blockIdx.x * 4 + wave;
    for (int i = threadIdx.x; i < 256; i += blockDim.x) s_lut[i] = o.lut[i];
    __syncthreads();
    if (q >= nq) return;   // no block-wide barrier below
    const int nc = (int)cv.n;
    const int nw = ((nc + 1) >> 1) + (((nc + 1) >> 1) & 1);
    uint32_t *votes = s_votes + (size_t)wave * nw;
    uint64_t *tab = reinterpret_cast<uint64_t *>(s_votes + (size_t)4 * nw) + (size_t)wave * o.rows * 4;
    for (int i = lane; i < nw; i += 64) votes[i] = 0u;
    for (int i = lane; i < o.rows * 4; i += 64) tab[i] = qv.peq[(size_t)q * o.rows * 4 + i];
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    const int64_t s0 = qv.off[q];
    const int plen = (int)(qv.off[q + 1] - s0);
    const uint8_t *str = qv.chars + s0;
    for (int p = lane; p + kQgram <= plen; p += 64) {
        const uint32_t b = qgram_bucket(str + p);
        const int e1 = cv.qg_off[b + 1];
        for (int e = cv.qg_off[b]; e < e1; e++) {
            const int r = cv.qg_cell[e];
            atomicAdd(&votes[r >> 1], (r & 1) ? 65536u : 1u);
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    int mine = -1;   // lane t < 4 takes the t-th best centre
    for (int t = 0; t < 4; t++) {
        uint64_t best = 0ull;   // (votes << 32) | ~rank: larger is better
        for (int i = lane; i < nw; i += 64) {
            const uint32_t v = votes[i];
            const uint64_t k0 = ((uint64_t)(v & 0xffffu) << 32) | (uint64_t)(0xffffffffu - (uint32_t)(2 * i));
            const uint64_t k1 = ((uint64_t)(v >> 16) << 32) | (uint64_t)(0xffffffffu - (uint32_t)(2 * i + 1));
            best = k0 > best ? k0 : best;
            best = k1 > best ? k1 : best;
        }
#pragma unroll
        for (int o2 = 32; o2 > 0; o2 >>= 1) {
            const uint64_t other = __shfl_xor(best, o2, 64);
            best = other > best ? other : best;
        }
        if ((best >> 32) == 0ull) break;   // wave-uniform
        const int r = (int)(0xffffffffu - (uint32_t)best);
        if (lane == t) mine = r;
        __builtin_amdgcn_wave_barrier();
        if (lane == 0) votes[r >> 1] &= (r & 1) ? 0x0000ffffu : 0xffff0000u;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    uint64_t key = ~0ull;   // (distance << 32) | rank: smaller is better
    if (mine >= 0) {
        const int32_t c0 = cv.off[mine];
        const int d = dev::myers_banded(static_cast<const uint64_t *>(tab), 4, plen, cv.chars + c0,
                                        cv.off[mine + 1] - c0, 63, static_cast<const uint8_t *>(s_lut));
        if (d <= 63) key = ((uint64_t)(uint32_t)d << 32) | (uint32_t)mine;
    }
#pragma unroll
    for (int o2 = 32; o2 > 0; o2 >>= 1) {
        const uint64_t other = __shfl_xor(key, o2, 64);
        key = other < key ? other : key;
    }
    if (lane == 0) {
        piv[q] = key == ~0ull ? -1 : (int32_t)(uint32_t)key;
        pivd[q] = key == ~0ull ? 0 : (int32_t)(key >> 32);
    }
}

void edit_pivot(const EditView &o, const QueryEdit &qv, int64_t nq, const CellView &cv, int32_t *piv,
                int32_t *pivd, hipStream_t st)
{
    if (nq == 0) return;
    require(cv.n > 0 && cv.n <= 4096 && cv.dist && cv.qg_off && cv.qg_cell, "edit_pivot: no centre tables");
    const int64_t nw = (cv.n + 1) / 2 + ((cv.n + 1) / 2) % 2;
    const size_t shm = (size_t)4 * nw * sizeof(uint32_t) + (size_t)4 * o.rows * 4 * sizeof(uint64_t);
    require(shm <= 65536, "edit_pivot: vote and table rows exceed the workgroup's LDS");
    hipLaunchKernelGGL(k_edit_pivot, dim3((unsigned)((nq + 3) / 4)), dim3(256), shm, st, o, qv, nq, cv, piv, pivd);
    check_launch(__func__);
}

// home[q] = the first cell (in chain order) on query q's list, n_cells when
// the list is empty, 0 when it overflowed.  One thread per query.
__global__ void k_first_cell(const int32_t *__restrict__ qcells, const int32_t *__restrict__ qcnt, int64_t n_cells,
                             int64_t nq, int32_t *__restrict__ home)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= nq) return;
    const int cnt = qcnt[q];
    int h = (int)n_cells;
    if (cnt > kQueryCells) h = 0;
    else
        for (int i = 0; i < cnt; i++) h = min(h, qcells[(size_t)q * kQueryCells + i]);
    home[q] = h;
}

void first_cell(const int32_t *qcells, const int32_t *qcnt, int64_t n_cells, int64_t nq, int32_t *home,
                hipStream_t st)
{
    if (nq == 0) return;
    hipLaunchKernelGGL(k_first_cell, dim3((unsigned)((nq + 255) / 256)), dim3(256), 0, st, qcells, qcnt, n_cells,
                       nq, home);
    check_launch(__func__);
}


void edit_cell_test(const EditView &o, const QueryEdit &qv, const int32_t *qlen, const float *QP, int mpad,
                    const float *T, int64_t nq, int max_qlen, const CellView &cv, const int32_t *piv,
                    const int32_t *pivd, int32_t *qcells, int32_t *qcnt, unsigned long long *counters,
                    const int32_t *order, hipStream_t st)
{
    if (nq == 0) return;
    fill_u32(reinterpret_cast<uint32_t *>(qcnt), nq, 0u, st);
    if (cv.n == 0) return;
    const int ntiles = (int)((nq + 63) / 64);
    const int W = std::max(1, (max_qlen + 63) / 64);
    const int64_t chunks = (cv.n + 255) / 256;
    const unsigned grid = (unsigned)(chunks * ntiles);
    const bool tab = (int64_t)o.rows * W * 64 <= kTileTabWords;
    const size_t shm = tab ? (size_t)o.rows * W * 64 * sizeof(uint64_t) : 0;
#define CT(WW, MP, TB)                                                                                            \
    hipLaunchKernelGGL((k_edit_cell_test<WW, MP, TB>), dim3(grid), dim3(256), shm, st, o, qv, qlen, QP, T, nq,    \
                       ntiles, cv, piv, pivd, qcells, qcnt, counters, order)
#define CTM(WW, TB)                 \
    if (mpad == 8) CT(WW, 8, TB);   \
    else if (mpad == 16) CT(WW, 16, TB); \
    else CT(WW, 32, TB);
#define CTW(TB)                     \
    switch (W) {                    \
    case 1: CTM(1, TB) break;       \
    case 2: CTM(2, TB) break;       \
    case 3: CTM(3, TB) break;       \
    default: CTM(4, TB) break;      \
    }
    if (tab) CTW(true) else CTW(false)
#undef CTW
#undef CTM
#undef CT
    check_launch(__func__);
}

void edit_leaf_ball(const EditView &o, const QueryEdit &qv, const int32_t *qlen, const int32_t *leaf_first,
                    const float *leafR, const int32_t *leaf_cell, const int32_t *cell_leaf, int64_t n_cells,
                    const int32_t *qcells, const int32_t *qcnt, const float *T, int64_t nq, int ntiles,
                    int max_qlen, uint64_t *leaf_mask, int32_t *items, uint32_t *item_count, int64_t item_cap,
                    int64_t n_leaves, hipStream_t st)
{
    fill_u32(reinterpret_cast<uint32_t *>(leaf_mask), n_leaves * ntiles * 2, 0u, st);
    if (nq == 0 || n_cells == 0) return;
    require(n_leaves < ((int64_t)1 << 31), "edit_leaf_ball: too many leaves");
    const int W = std::max(1, (max_qlen + 63) / 64);
    const unsigned grid = (unsigned)((nq + 3) / 4);
    const size_t shm = (size_t)4 * o.rows * 4 * sizeof(uint64_t);
    auto *lm = reinterpret_cast<unsigned long long *>(leaf_mask);
#define EQ(WW)                                                                                                 \
    hipLaunchKernelGGL(k_edit_leaf_query<WW>, dim3(grid), dim3(256), shm, st, o, qv, qlen, T, leaf_first, leafR, \
                       leaf_cell, cell_leaf, n_cells, n_leaves, qcells, qcnt, nq, ntiles, lm, items, item_count,  \
                       item_cap)
    switch (W) {
    case 1: EQ(1); break;
    case 2: EQ(2); break;
    case 3: EQ(3); break;
    default: EQ(4); break;
    }
#undef EQ
    check_launch(__func__);
}

}  // namespace k
}  // namespace gts
