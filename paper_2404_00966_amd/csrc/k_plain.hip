// The plain form: one query per workgroup runs every stage of the search
// itself -- query-to-pivot distances, the layer-by-layer child test over the
// node table (Algorithm 4's frontier, compacted with wave ballots), Lemma 1
// on every object of the surviving leaves, and exact verification.  It emits
// verified (query, key) entries; ordering and CSR assembly are shared with
// the batched form.
#include "dev_common.h"
#include "gts_internal.h"
#include "kernels.h"

namespace gts {
namespace k {


constexpr int kPlainCand = 1024;
constexpr int kPlainBlock = 256;

// Compact `pass` lanes of the workgroup into buf (counter in LDS).
__device__ __forceinline__ void block_push(bool pass, int32_t val, int32_t *buf, int *counter)
{
    const uint64_t b = dev::ballot(pass);
    int base = 0;
    if (dev::lane_id() == 0 && b) base = atomicAdd(counter, __popcll(b));
    base = __shfl(base, 0, 64);
    if (pass) buf[base + dev::lanes_below(b)] = val;
}

// Layer-by-layer child test from the root to the leaves; returns the buffer
// whose first *s_nf entries are the surviving leaves' node ids.
template <int MP>
__device__ int32_t *tree_frontier(const TreeView &t, const float *s_qp, float thr, int32_t *fr0, int32_t *fr1,
                                  int *s_nf, long long *tests)
{
    if (threadIdx.x == 0) {
        fr0[0] = 0;
        *s_nf = 1;
    }
    __syncthreads();
    int32_t *cur = fr0, *nxt = fr1;
    for (int l = 1; l <= t.levels; l++) {
        const int nf = *s_nf;
        __syncthreads();
        if (threadIdx.x == 0) *s_nf = 0;
        __syncthreads();
        const int total = nf * t.fanout;
        for (int i0 = 0; i0 < total; i0 += blockDim.x) {
            const int i = i0 + threadIdx.x;
            bool pass = false;
            int32_t child = 0;
            if (i < total) {
                child = cur[i / t.fanout] * t.fanout + 1 + i % t.fanout;
                float g = -INFINITY;
#pragma unroll
                for (int p = 0; p < MP; p++) {
                    const float lo = t.box_lo[(size_t)p * t.n_nodes + child];
                    const float hi = t.box_hi[(size_t)p * t.n_nodes + child];
                    g = fmaxf(g, fmaxf(lo - s_qp[p], s_qp[p] - hi));
                }
                pass = g <= thr;
                (*tests)++;
            }
            block_push(pass, child, nxt, s_nf);
        }
        __syncthreads();
        int32_t *tmp = cur;
        cur = nxt;
        nxt = tmp;
    }
    return cur;
}

__device__ __forceinline__ void emit_verified(const PlainArgs &a, int64_t q, uint32_t dbits, uint32_t id)
{
    const CandCount idx = atomicAdd(a.out_count, (CandCount)1);
    if ((int64_t)idx < a.out_cap) {
        Cand cd;
        cd.q = (int32_t)q;
        cd.pos = -1;
        cd.val = ((uint64_t)dbits << 32) | id;
        a.out[idx] = cd;
    }
}

// ---------------------------------------------------------------------------
// L2
// ---------------------------------------------------------------------------
// cut: the emission cutoff -- the radius for range queries; for kNN queries
// the bound widened to cover any float32 summation order (the final top-k
// is taken when the answers are sorted).
template <bool L1>
__device__ void plain_flush_l2(const L2View &o, const PlainArgs &a, int64_t q, const float *qrow, float cut,
                               const int32_t *s_cand, int nc, long long *verified)
{
    const int grp = threadIdx.x >> 4, sl = threadIdx.x & 15;
    for (int c0 = 0; c0 < nc; c0 += kPlainBlock / 16) {
        const int c = c0 + grp;
        float acc = 0.f;
        int32_t p = 0;
        if (c < nc) {
            p = s_cand[c];
            const float *x = o.X32 + (size_t)p * o.dp;
            for (int d = sl; d < o.dp; d += 16) acc = dev::dterm<L1>(acc, qrow[d], x[d]);
        }
#pragma unroll
        for (int off = 8; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 16);
        if (sl == 0 && c < nc) {
            (*verified)++;
            const float d = dev::dfinish<L1>(acc);
            if (d <= cut) emit_verified(a, q, __float_as_uint(dev::out_dist(d, a.angular != 0)), a.ids[p]);
        }
    }
}

template <int MP, bool L1>
__global__ __launch_bounds__(kPlainBlock) void k_plain_l2(TreeView t, L2View o, const float *__restrict__ P32,
                                                          int m, const float *__restrict__ PT,
                                                          const float *__restrict__ Q32, PlainArgs a)
{
    __shared__ float s_qp[MP];
    __shared__ int32_t s_cand[kPlainCand];
    __shared__ int s_nc, s_nf;
    int32_t *fr0 = a.frontier + (size_t)blockIdx.x * 2 * t.n_leaves;
    int32_t *fr1 = fr0 + t.n_leaves;
    long long tests = 0, verified = 0, leaves = 0;
    for (int64_t q = blockIdx.x; q < a.nq; q += gridDim.x) {
        const float *qrow = Q32 + (size_t)q * o.dp;
        if (threadIdx.x < MP) {
            float acc = 0.f;
            if ((int)threadIdx.x < m) {
                const float *p = P32 + (size_t)threadIdx.x * o.dp;
                float a0 = 0.f, a1 = 0.f, a2 = 0.f, a3 = 0.f;
                for (int c = 0; c < o.dp; c += 4) {
                    a0 = dev::dterm<L1>(a0, qrow[c], p[c]);
                    a1 = dev::dterm<L1>(a1, qrow[c + 1], p[c + 1]);
                    a2 = dev::dterm<L1>(a2, qrow[c + 2], p[c + 2]);
                    a3 = dev::dterm<L1>(a3, qrow[c + 3], p[c + 3]);
                }
                acc = dev::dfinish<L1>((a0 + a1) + (a2 + a3));
            }
            s_qp[threadIdx.x] = acc;
        }
        if (threadIdx.x == 0) s_nc = 0;
        __syncthreads();
        const float base = a.base[q];
        float qmax = 0.f;
        for (int p = 0; p < MP; p++) qmax = fmaxf(qmax, s_qp[p]);
        const float T = base * (1.f + 2.f * a.delta);
        const float thr = T + 2.f * a.delta * (qmax + a.pt_max);
        const float cut = a.kq[q] > 0 ? T : base;
        int32_t *lv = tree_frontier<MP>(t, s_qp, thr, fr0, fr1, &s_nf, &tests);
        int nf = s_nf;
        if (a.leaf_piv32) {
            // Lemma 1 with each surviving leaf's own pivot: the leaf is kept
            // unless d(q, p_L) - R_L > T (16 lanes per leaf pivot distance)
            int32_t *other = lv == fr0 ? fr1 : fr0;
            __syncthreads();
            if (threadIdx.x == 0) s_nf = 0;
            __syncthreads();
            const int grp = threadIdx.x >> 4, sl = threadIdx.x & 15;
            for (int e0 = 0; e0 < nf; e0 += kPlainBlock / 16) {
                const int e = e0 + grp;
                const int32_t node = e < nf ? lv[e] : 0;
                float acc = 0.f;
                if (e < nf) {
                    const float *pv = a.leaf_piv32 + (size_t)(node - t.leaf0) * o.dp;
                    for (int dd = sl; dd < o.dp; dd += 16) acc = dev::dterm<L1>(acc, qrow[dd], pv[dd]);
                }
#pragma unroll
                for (int off = 8; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 16);
                bool pass = false;
                if (e < nf) pass = dev::dfinish<L1>(acc) * (1.f - 2.f * a.delta) - a.leafR[node - t.leaf0] <= T;
                block_push(sl == 0 && pass, node, other, &s_nf);
            }
            __syncthreads();
            nf = s_nf;
            lv = other;
        }
        leaves += nf;
        for (int e = 0; e < nf; e++) {
            const int64_t leaf = lv[e] - t.leaf0;
            const int p0 = t.leaf_first[leaf];
            const int cnt = t.leaf_cnt[leaf];
            for (int j0 = 0; j0 < cnt; j0 += kPlainBlock) {
                __syncthreads();
                const int nc = s_nc;
                if (nc + kPlainBlock > kPlainCand) {
                    plain_flush_l2<L1>(o, a, q, qrow, cut, s_cand, nc, &verified);
                    __syncthreads();
                    if (threadIdx.x == 0) s_nc = 0;
                    __syncthreads();
                }
                // Lemma 1 on every pivot for this object
                const int j = j0 + threadIdx.x;
                const int p = p0 + j;
                bool pass = false;
                if (j < cnt && !((a.tomb[p >> 5] >> (p & 31)) & 1u)) {
                    float lb = 0.f;
#pragma unroll
                    for (int i = 0; i < MP; i++) lb = fmaxf(lb, fabsf(s_qp[i] - PT[(size_t)i * o.n + p]));
                    pass = lb <= thr;
                }
                block_push(pass, p, s_cand, &s_nc);
            }
        }
        __syncthreads();
        plain_flush_l2<L1>(o, a, q, qrow, cut, s_cand, s_nc, &verified);
        __syncthreads();
    }
    if (threadIdx.x % 16 == 0 && verified) count_add(a.counters, CNT_VERIFIED, (unsigned long long)verified);
    if (threadIdx.x == 0 && leaves) count_add(a.counters, CNT_LEAF_PAIRS, (unsigned long long)leaves);
    if (tests) count_add(a.counters, CNT_NODE_TESTS, (unsigned long long)tests);
}

void plain_l2(const TreeView &t, const L2View &o, const float *P32, int m, const float *PT, const float *Q32,
              const PlainArgs &a, hipStream_t st)
{
    if (a.nq == 0) return;
#define PL(MP, L1) \
    hipLaunchKernelGGL((k_plain_l2<MP, L1>), dim3((unsigned)a.grid), dim3(kPlainBlock), 0, st, t, o, P32, m, PT, Q32, a)
    if (a.l1) {
        if (t.mpad == 8) PL(8, true);
        else if (t.mpad == 16) PL(16, true);
        else PL(32, true);
    } else {
        if (t.mpad == 8) PL(8, false);
        else if (t.mpad == 16) PL(16, false);
        else PL(32, false);
    }
#undef PL
    check_launch(__func__);
}

// ---------------------------------------------------------------------------
// EDIT: the query is the Myers pattern throughout (its match table in LDS);
// pivots and objects are texts.
// ---------------------------------------------------------------------------
__device__ void plain_flush_edit(const EditView &o, const PlainArgs &a, int64_t q, const uint64_t *s_peq, int plen,
                                 int cut, const int32_t *s_cand, int nc, long long *verified, const uint8_t *s_lut)
{
    for (int c = threadIdx.x; c < nc; c += blockDim.x) {
        const int32_t p = s_cand[c];
        const int32_t s0 = o.soff[p];
        const int tl = o.soff[p + 1] - s0;
        (*verified)++;
        const int d = dev::myers_any(s_peq, plen, o.chars + s0, tl, cut, s_lut);
        if (d <= cut) emit_verified(a, q, (uint32_t)d, a.ids[p]);
    }
}

template <int MP>
__global__ __launch_bounds__(kPlainBlock) void k_plain_edit(TreeView t, EditView o, const uint8_t *__restrict__ pchars,
                                                            const int32_t *__restrict__ poff, int m,
                                                            const uint8_t *__restrict__ PTe, QueryEdit qv,
                                                            PlainArgs a)
{
    __shared__ uint64_t s_peq[257 * 4];
    __shared__ uint8_t s_lut[256];
    __shared__ float s_qp[MP];
    __shared__ int32_t s_cand[kPlainCand];
    __shared__ int s_nc, s_nf;
    int32_t *fr0 = a.frontier + (size_t)blockIdx.x * 2 * t.n_leaves;
    int32_t *fr1 = fr0 + t.n_leaves;
    long long tests = 0, verified = 0, leaves = 0;
    for (int64_t q = blockIdx.x; q < a.nq; q += gridDim.x) {
        const int64_t qa = qv.off[q];
        const int plen = (int)(qv.off[q + 1] - qa);
        for (int i = threadIdx.x; i < o.rows * 4; i += blockDim.x) s_peq[i] = 0ull;
        for (int i = threadIdx.x; i < 256; i += blockDim.x) s_lut[i] = o.lut[i];
        __syncthreads();
        dev::peq_fill(s_peq, qv.chars + qa, plen, s_lut, o.rows);
        if (threadIdx.x == 0) s_nc = 0;
        __syncthreads();
        if (threadIdx.x < MP) {
            int d = 0;
            if ((int)threadIdx.x < m) {
                const int32_t s0 = poff[threadIdx.x];
                d = dev::myers_any(s_peq, plen, pchars + s0, poff[threadIdx.x + 1] - s0, 1 << 30, s_lut);
            }
            s_qp[threadIdx.x] = (float)d;
        }
        __syncthreads();
        const int cut = (int)floorf(fminf(a.base[q], 1e6f));
        int32_t *lv = tree_frontier<MP>(t, s_qp, (float)cut, fr0, fr1, &s_nf, &tests);
        const int nf = s_nf;
        leaves += nf;
        for (int e = 0; e < nf; e++) {
            const int64_t leaf = lv[e] - t.leaf0;
            const int p0 = t.leaf_first[leaf];
            const int cnt = t.leaf_cnt[leaf];
            for (int j0 = 0; j0 < cnt; j0 += kPlainBlock) {
                __syncthreads();
                const int nc = s_nc;
                if (nc + kPlainBlock > kPlainCand) {
                    plain_flush_edit(o, a, q, s_peq, plen, cut, s_cand, nc, &verified, s_lut);
                    __syncthreads();
                    if (threadIdx.x == 0) s_nc = 0;
                    __syncthreads();
                }
                const int j = j0 + threadIdx.x;
                const int p = p0 + j;
                bool pass = false;
                if (j < cnt && !((a.tomb[p >> 5] >> (p & 31)) & 1u)) {
                    const int olen = o.soff[p + 1] - o.soff[p];
                    pass = abs(olen - plen) <= cut;
#pragma unroll
                    for (int i = 0; i < MP; i++)
                        pass = pass && fabsf(s_qp[i] - (float)PTe[(size_t)i * o.n + p]) <= (float)cut;
                }
                block_push(pass, p, s_cand, &s_nc);
            }
        }
        __syncthreads();
        plain_flush_edit(o, a, q, s_peq, plen, cut, s_cand, s_nc, &verified, s_lut);
        __syncthreads();
    }
    if (verified) count_add(a.counters, CNT_VERIFIED, (unsigned long long)verified);
    if (threadIdx.x == 0 && leaves) count_add(a.counters, CNT_LEAF_PAIRS, (unsigned long long)leaves);
    if (tests) count_add(a.counters, CNT_NODE_TESTS, (unsigned long long)tests);
}

void plain_edit(const TreeView &t, const EditView &o, const uint8_t *pchars, const int32_t *poff, int m,
                const uint8_t *PTe, const QueryEdit &qv, const PlainArgs &a, hipStream_t st)
{
    if (a.nq == 0) return;
#define PE(MP)                                                                                                \
    hipLaunchKernelGGL(k_plain_edit<MP>, dim3((unsigned)a.grid), dim3(kPlainBlock), 0, st, t, o, pchars, poff, m, \
                       PTe, qv, a)
    if (t.mpad == 8) PE(8);
    else if (t.mpad == 16) PE(16);
    else PE(32);
#undef PE
    check_launch(__func__);
}

}  // namespace k
}  // namespace gts
