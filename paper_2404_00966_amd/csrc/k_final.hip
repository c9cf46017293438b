// Candidate grouping by query, exact verification with per-query selection
// and (distance, id) ordering, and CSR assembly.
#include "dev_common.h"
#include "gts_internal.h"
#include "kernels.h"

namespace gts {
namespace k {


// Runs of equal query among a wave's 64 consecutive candidates (the sweep
// writes each lane's hits of one tile next to each other): the first lane of
// a run makes one atomic for the whole run.  *head_lane = first lane of this
// lane's run; returns the run length at its first lane, 0 elsewhere.
__device__ __forceinline__ int query_run(int32_t q, bool valid, int *head_lane)
{
    const int lane = dev::lane_id();
    const int32_t prev = __shfl_up(q, 1, 64);
    const bool head = valid && (lane == 0 || prev != q);
    // both ballots by the whole wave, before any lane leaves
    const uint64_t hm = dev::ballot(head);
    const int nvalid = __popcll(dev::ballot(valid));          // valid lanes form a prefix
    const uint64_t upto = lane == 63 ? ~0ull : ((2ull << lane) - 1ull);
    *head_lane = 63 - __clzll((long long)(hm & upto));
    if (!head) return 0;
    const uint64_t after = hm & ~upto;
    const int end = after ? __ffsll((long long)after) - 1 : nvalid;
    return end - lane;
}

__global__ __launch_bounds__(256) void k_group_hist(const Cand *__restrict__ c, const uint32_t *__restrict__ count,
                                                    int64_t cap, uint32_t *__restrict__ qcount)
{
    int64_t n = *count;
    if (n > cap) n = cap;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t b0 = (int64_t)blockIdx.x * blockDim.x + (threadIdx.x & ~63u); b0 < n; b0 += stride) {
        const int64_t i = b0 + dev::lane_id();
        const bool valid = i < n;
        const int32_t q = valid ? c[i].q : -1;
        int hl;
        const int len = query_run(q, valid, &hl);
        if (len) atomicAdd(&qcount[q], (uint32_t)len);
    }
}

void group_hist(const Cand *c, const uint32_t *count, int64_t cap, uint32_t *qcount, hipStream_t st)
{
    hipLaunchKernelGGL(k_group_hist, dim3(2048), dim3(256), 0, st, c, count, cap, qcount);
    check_launch(__func__);
}

// Exclusive scan of n counts into out[0..n], one workgroup of 1024 threads.
__global__ __launch_bounds__(1024) void k_scan_u32(const uint32_t *__restrict__ in, int64_t n,
                                                   int64_t *__restrict__ out)
{
    __shared__ int64_t s[1024];
    const int t = threadIdx.x;
    const int64_t per = (n + 1023) / 1024;
    const int64_t a = (int64_t)t * per;
    const int64_t b = a + per < n ? a + per : n;
    int64_t sum = 0;
    for (int64_t i = a; i < b; i++) sum += in[i];
    s[t] = sum;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        int64_t v = t >= off ? s[t - off] : 0;
        __syncthreads();
        s[t] += v;
        __syncthreads();
    }
    int64_t run = s[t] - sum;
    for (int64_t i = a; i < b; i++) {
        out[i] = run;
        run += in[i];
    }
    if (t == 1023) out[n] = s[1023];
}

void scan_u32(const uint32_t *in, int64_t n, int64_t *out, hipStream_t st)
{
    hipLaunchKernelGGL(k_scan_u32, dim3(1), dim3(1024), 0, st, in, n, out);
    check_launch(__func__);
}

__global__ __launch_bounds__(256) void k_group_scatter(const Cand *__restrict__ c, const uint32_t *__restrict__ count,
                                                       int64_t cap, const int64_t *__restrict__ qoff,
                                                       uint32_t *__restrict__ cursor, Cand *__restrict__ grouped)
{
    int64_t n = *count;
    if (n > cap) n = cap;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int lane = dev::lane_id();
    for (int64_t b0 = (int64_t)blockIdx.x * blockDim.x + (threadIdx.x & ~63u); b0 < n; b0 += stride) {
        const int64_t i = b0 + lane;
        const bool valid = i < n;
        Cand cd;
        cd.q = -1;
        if (valid) cd = c[i];
        int hl;
        const int len = query_run(cd.q, valid, &hl);
        uint32_t base = 0;
        if (len) base = atomicAdd(&cursor[cd.q], (uint32_t)len);
        base = __shfl(base, hl, 64);
        if (valid) grouped[qoff[cd.q] + base + (uint32_t)(lane - hl)] = cd;
    }
}

void group_scatter(const Cand *c, const uint32_t *count, int64_t cap, const int64_t *qoff, uint32_t *cursor,
                   Cand *grouped, hipStream_t st)
{
    hipLaunchKernelGGL(k_group_scatter, dim3(2048), dim3(256), 0, st, c, count, cap, qoff, cursor, grouped);
    check_launch(__func__);
}

// Sort the keys of one query (in LDS or, for a large segment, in its
// power-of-two scratch run) and write the first `keep` to out.
__device__ void sort_and_emit(uint64_t *keys, int nk, int64_t cap, int k, uint64_t *out, uint32_t *out_count_q)
{
    const int P = dev::next_pow2(nk > 1 ? nk : 1);
    for (int i = nk + threadIdx.x; i < P && i < cap; i += blockDim.x) keys[i] = ~0ull;
    dev::bitonic_sort(keys, P);
    const int nout = (k > 0 && k < nk) ? k : nk;
    for (int j = threadIdx.x; j < nout; j += blockDim.x) out[j] = keys[j];
    if (threadIdx.x == 0) *out_count_q = (uint32_t)nout;
}

// ---------------------------------------------------------------------------
// L2: per query, one workgroup.  kNN queries first keep only candidates
// whose distance interval can reach the k smallest upper bounds: from the
// bf16 estimate e of d^2, d lies in [sqrt(e - eps) - eq - ex,
// sqrt(e + eps) + eq + ex].  Then each kept candidate gets its exact float32
// distance (direct difference, 16 lanes per candidate); range queries keep
// d <= r, kNN queries keep everything; keys are sorted by (d, id).
// ---------------------------------------------------------------------------
__device__ __forceinline__ void l2_interval(const Cand &c, float qnn, float qerr, const L2View &o, float eps_a,
                                            float eps_b, float eps_c, float delta, float *lo, float *hi)
{
    if (c.pos < 0) {
        const float d = __uint_as_float((uint32_t)(c.val >> 32));
        *lo = d * (1.f - 2.f * delta);
        *hi = d * (1.f + 2.f * delta);
        return;
    }
    const float est = __uint_as_float((uint32_t)c.val);
    const float xnn = o.xn[c.pos];
    const float eps = eps_a * (qnn + xnn) + eps_b * sqrtf(qnn * xnn) + eps_c * fabsf(est);
    const float err = qerr + o.xe[c.pos];
    *hi = sqrtf(fmaxf(est + eps, 0.f)) + err;
    *lo = sqrtf(fmaxf(est - eps, 0.f)) - err;
}

// One workgroup for query q (its candidates more than one wave verifies):
// kNN interval selection by a sort of the upper ends, rechecks by 16-lane
// groups, keys sorted in LDS (s_keys, kSortCap) or in the query's scratch run.
__device__ void verify_l2_block(const VerifyArgs &a, const L2View &o, const QueryL2 &qv, float delta, float eps_a,
                                float eps_b, float eps_c, int64_t q, uint64_t *s_keys)
{
    __shared__ int s_n;
    __shared__ float s_ub;
    const int64_t seg0 = a.qoff[q];
    const int ns = (int)(a.qoff[q + 1] - seg0);
    const int k = a.kq ? a.kq[q] : 0;
    const float base = a.base[q];
    const int64_t boff = a.big_off ? a.big_off[q] : -1;
    const bool big = boff >= 0;
    uint64_t *keys = big ? a.scratch + boff : s_keys;
    const int64_t cap = big ? dev::next_pow2(ns) : kSortCap;
    const float qnn = qv.qn[q];
    const float qerr = qv.qe[q];
    const Cand *g = a.grouped + seg0;

    if (threadIdx.x == 0) {
        s_n = 0;
        s_ub = INFINITY;
    }
    if (k > 0 && ns > k && !big) {
        for (int i = threadIdx.x; i < ns; i += blockDim.x) {
            float lo, hi;
            l2_interval(g[i], qnn, qerr, o, eps_a, eps_b, eps_c, delta, &lo, &hi);
            s_keys[i] = (uint64_t)__float_as_uint(hi);
        }
        const int P = dev::next_pow2(ns);
        for (int i = ns + threadIdx.x; i < P; i += blockDim.x) s_keys[i] = ~0ull;
        dev::bitonic_sort(s_keys, P);
        if (threadIdx.x == 0) s_ub = __uint_as_float((uint32_t)s_keys[k - 1]) * (1.f + 4.f * delta);
    }
    __syncthreads();
    const float ub = s_ub;
    const int grp = threadIdx.x >> 4, sl = threadIdx.x & 15;
    const float *qrow = qv.Q32 + (size_t)q * o.dp;
    long long verified = 0;
    // two candidates per 16-lane group and step, both rows in flight together
    auto emit = [&](bool valid, const Cand &c, bool need, float acc) {
        if (sl != 0 || !valid) return;
        bool keep = false;
        uint64_t key = 0;
        if (c.pos < 0) {
            keep = true;
            key = c.val;
        } else if (need) {
            verified++;
            const float d = sqrtf(acc);
            keep = k > 0 || d <= base;
            key = ((uint64_t)__float_as_uint(d) << 32) | a.ids[c.pos];
        }
        if (keep) {
            const int slot = atomicAdd(&s_n, 1);
            keys[slot] = key;
        }
    };
    auto needs = [&](bool valid, const Cand &c) {
        bool need = valid && c.pos >= 0;
        if (need && k > 0 && ub < INFINITY) {
            float lo, hi;
            l2_interval(c, qnn, qerr, o, eps_a, eps_b, eps_c, delta, &lo, &hi);
            need = lo <= ub;
        }
        return need;
    };
    for (int i0 = 0; i0 < ns; i0 += 32) {
        const int ia = i0 + grp, ib = i0 + 16 + grp;
        const bool va = ia < ns, vb = ib < ns;
        Cand ca, cb;
        ca.q = cb.q = 0;
        ca.pos = cb.pos = -1;
        ca.val = cb.val = 0;
        if (va) ca = g[ia];
        if (vb) cb = g[ib];
        const bool na = needs(va, ca), nb = needs(vb, cb);
        const float *xa = na ? o.X32 + (size_t)ca.pos * o.dp : qrow;
        const float *xb = nb ? o.X32 + (size_t)cb.pos * o.dp : qrow;
        float acca = 0.f, accb = 0.f;
        if (na || nb) {
            for (int d = sl; d < o.dp; d += 16) {
                const float qd = qrow[d];
                const float dfa = qd - xa[d];
                const float dfb = qd - xb[d];
                acca = fmaf(dfa, dfa, acca);
                accb = fmaf(dfb, dfb, accb);
            }
        }
#pragma unroll
        for (int off = 8; off > 0; off >>= 1) {
            acca += __shfl_xor(acca, off, 16);
            accb += __shfl_xor(accb, off, 16);
        }
        emit(va, ca, na, acca);
        emit(vb, cb, nb, accb);
    }
    __syncthreads();
    if (threadIdx.x % 16 == 0 && verified) atomicAdd(&a.counters[CNT_VERIFIED], (unsigned long long)verified);
    const int nk = s_n;
    sort_and_emit(keys, nk, cap, k, a.out_keys + seg0, a.out_count + q);
}

// Bitonic sort of n (a power of two) keys in LDS by one wave (lanes in
// lockstep: a wave barrier orders the passes).
__device__ void wave_bitonic_sort(uint64_t *a, int n)
{
    const int lane = threadIdx.x & 63;
    for (int size = 2; size <= n; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            for (int i = lane; i < (n >> 1); i += 64) {
                const int lo = 2 * i - (i & (stride - 1));
                const int hi = lo + stride;
                const bool up = (lo & size) == 0;
                const uint64_t x = a[lo], y = a[hi];
                if ((x > y) == up) {
                    a[lo] = y;
                    a[hi] = x;
                }
            }
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// One wave for query q (at most kWaveSortCap candidates).  kNN: the k-th
// smallest upper interval end over the candidates, found by a 32-step
// binary search over the float bits (counting with ballots), bounds the
// answer set; only candidates whose lower end can reach it are rechecked.
// Rechecks: 16 lanes per candidate, two candidates per group in flight, the
// same strided float32 sum as every other exact L2 distance here.  Kept keys
// are compacted with ballots into the wave's LDS run and sorted there.
__device__ void verify_l2_wave(const VerifyArgs &a, const L2View &o, const QueryL2 &qv, float delta, float eps_a,
                               float eps_b, float eps_c, int64_t q, uint64_t *keys)
{
    const int lane = threadIdx.x & 63;
    const int64_t seg0 = a.qoff[q];
    const int ns = (int)(a.qoff[q + 1] - seg0);
    const int k = a.kq ? a.kq[q] : 0;
    const float base = a.base[q];
    const float qnn = qv.qn[q];
    const float qerr = qv.qe[q];
    const Cand *g = a.grouped + seg0;
    float ub = INFINITY;
    if (k > 0 && ns > k) {
        for (int i = lane; i < ns; i += 64) {
            float lo, hi;
            l2_interval(g[i], qnn, qerr, o, eps_a, eps_b, eps_c, delta, &lo, &hi);
            keys[i] = __float_as_uint(hi);
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        // smallest v with #{hi <= v} >= k (hi >= 0, so float order = bit order)
        uint32_t lo_v = 0u, hi_v = 0xffffffffu;
        while (lo_v < hi_v) {
            const uint32_t mid = lo_v + ((hi_v - lo_v) >> 1);
            int c = 0;
            for (int i0 = 0; i0 < ns; i0 += 64) {
                const int i = i0 + lane;
                c += __popcll(dev::ballot(i < ns && (uint32_t)keys[i] <= mid));
            }
            if (c >= k) hi_v = mid;
            else lo_v = mid + 1u;
        }
        ub = __uint_as_float(lo_v) * (1.f + 4.f * delta);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    const int grp = lane >> 4, sl = lane & 15;
    const float *qrow = qv.Q32 + (size_t)q * o.dp;
    long long verified = 0;
    int nk = 0;
    for (int i0 = 0; i0 < ns; i0 += 8) {
        const int ia = i0 + grp, ib = i0 + 4 + grp;
        const bool va = ia < ns, vb = ib < ns;
        Cand ca, cb;
        ca.q = cb.q = 0;
        ca.pos = cb.pos = -1;
        ca.val = cb.val = 0;
        if (va) ca = g[ia];
        if (vb) cb = g[ib];
        bool na = va && ca.pos >= 0, nb = vb && cb.pos >= 0;
        if (k > 0 && ub < INFINITY) {
            float lo, hi;
            if (na) {
                l2_interval(ca, qnn, qerr, o, eps_a, eps_b, eps_c, delta, &lo, &hi);
                na = lo <= ub;
            }
            if (nb) {
                l2_interval(cb, qnn, qerr, o, eps_a, eps_b, eps_c, delta, &lo, &hi);
                nb = lo <= ub;
            }
        }
        const float *xa = na ? o.X32 + (size_t)ca.pos * o.dp : qrow;
        const float *xb = nb ? o.X32 + (size_t)cb.pos * o.dp : qrow;
        float acca = 0.f, accb = 0.f;
        if (na || nb) {
            for (int d = sl; d < o.dp; d += 16) {
                const float qd = qrow[d];
                const float dfa = qd - xa[d];
                const float dfb = qd - xb[d];
                acca = fmaf(dfa, dfa, acca);
                accb = fmaf(dfb, dfb, accb);
            }
        }
#pragma unroll
        for (int off = 8; off > 0; off >>= 1) {
            acca += __shfl_xor(acca, off, 16);
            accb += __shfl_xor(accb, off, 16);
        }
        auto decide = [&](bool valid, const Cand &c, bool need, float acc, uint64_t *key) {
            if (!valid) return false;
            if (c.pos < 0) {
                *key = c.val;
                return true;
            }
            if (!need) return false;
            verified++;
            const float d = sqrtf(acc);
            *key = ((uint64_t)__float_as_uint(d) << 32) | a.ids[c.pos];
            return k > 0 || d <= base;
        };
        uint64_t ka = 0, kb = 0;
        const bool keepa = sl == 0 && decide(va, ca, na, acca, &ka);
        const bool keepb = sl == 0 && decide(vb, cb, nb, accb, &kb);
        const uint64_t ma = dev::ballot(keepa), mb = dev::ballot(keepb);
        if (keepa) keys[nk + dev::lanes_below(ma)] = ka;
        nk += __popcll(ma);
        if (keepb) keys[nk + dev::lanes_below(mb)] = kb;
        nk += __popcll(mb);
    }
    for (int o2 = 32; o2 > 0; o2 >>= 1) verified += __shfl_xor(verified, o2, 64);
    if (lane == 0 && verified) atomicAdd(&a.counters[CNT_VERIFIED], (unsigned long long)verified);
    const int P = dev::next_pow2(nk > 1 ? nk : 1);
    for (int i = nk + lane; i < P; i += 64) keys[i] = ~0ull;
    wave_bitonic_sort(keys, P);
    const int nout = (k > 0 && k < nk) ? k : nk;
    for (int j = lane; j < nout; j += 64) a.out_keys[seg0 + j] = keys[j];
    if (lane == 0) a.out_count[q] = (uint32_t)nout;
}

// One launch for both forms: workgroups [0, n_blk) take the queries of
// blk_q (more than kWaveSortCap candidates) one each, the rest take four
// queries each, one per wave, skipping those; the long workgroups start first
// and overlap the bulk of the work.
__global__ __launch_bounds__(256) void k_verify_l2(VerifyArgs a, L2View o, QueryL2 qv, float delta, float eps_a,
                                                   float eps_b, float eps_c, const int32_t *__restrict__ blk_q,
                                                   int n_blk)
{
    __shared__ uint64_t s_mem[kSortCap];
    static_assert(4 * kWaveSortCap <= kSortCap, "wave runs must fit the workgroup's LDS");
    if ((int)blockIdx.x < n_blk) {
        verify_l2_block(a, o, qv, delta, eps_a, eps_b, eps_c, blk_q[blockIdx.x], s_mem);
        return;
    }
    // wave mode: past the workgroup-mode blocks (rounded up to 8), XCD x
    // takes the x-th contiguous eighth of the 4-query blocks
    const int wave = threadIdx.x >> 6;
    const int nb8 = (n_blk + 7) & ~7;
    if ((int)blockIdx.x < nb8) return;
    const int64_t w = blockIdx.x - nb8, per = (gridDim.x - nb8) >> 3;
    const int64_t q = ((w & 7) * per + (w >> 3)) * 4 + wave;
    if (q >= a.nq) return;
    const int ns = (int)(a.qoff[q + 1] - a.qoff[q]);
    if (ns > kWaveSortCap) return;
    verify_l2_wave(a, o, qv, delta, eps_a, eps_b, eps_c, q, s_mem + wave * kWaveSortCap);
}

void verify_l2(const VerifyArgs &a, const L2View &o, const QueryL2 &qv, float delta, const int32_t *blk_q, int n_blk,
               hipStream_t st)
{
    if (a.nq == 0) return;
    const float u = 5.9604645e-8f;
    const int D = o.ksteps * 32;
    const float eps_a = 2.f * (D + 8) * u, eps_b = 2.f * (4 * D + 8) * u, eps_c = 8.f * u;
    const unsigned grid = (unsigned)(((n_blk + 7) & ~7) + ((a.nq + 3) / 4 + 7) / 8 * 8);
    hipLaunchKernelGGL(k_verify_l2, dim3(grid), dim3(256), 0, st, a, o, qv, delta, eps_a, eps_b, eps_c, blk_q, n_blk);
    check_launch(__func__);
}

// ---------------------------------------------------------------------------
// EDIT: per query, one workgroup; the query's match table sits in LDS and
// every lane verifies one candidate (object string as the text) with the
// early-exit cutoff floor(base); kept keys are sorted by (d, id).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_verify_edit(VerifyArgs a, EditView o, QueryEdit qv)
{
    __shared__ uint64_t s_keys[kSortCap];
    __shared__ uint64_t s_peq[257 * 4];
    __shared__ uint8_t s_lut[256];
    __shared__ int s_n;
    // gridDim.x is a multiple of 8: XCD x takes the x-th contiguous eighth of
    // the queries, whose neighbours share candidates in that XCD's L2
    const int64_t per = gridDim.x >> 3;
    const int64_t q = (int64_t)(blockIdx.x & 7) * per + (blockIdx.x >> 3);
    if (q >= a.nq) return;
    const int64_t seg0 = a.qoff[q];
    const int ns = (int)(a.qoff[q + 1] - seg0);
    const int k = a.kq ? a.kq[q] : 0;
    const int cut = (int)floorf(fminf(a.base[q], 1e6f));
    const int64_t boff = a.big_off ? a.big_off[q] : -1;
    const bool big = boff >= 0;
    uint64_t *keys = big ? a.scratch + boff : s_keys;
    const int64_t cap = big ? dev::next_pow2(ns) : kSortCap;
    const Cand *g = a.grouped + seg0;
    const uint64_t *pq = qv.peq + (size_t)q * o.rows * 4;
    for (int i = threadIdx.x; i < o.rows * 4; i += blockDim.x) s_peq[i] = pq[i];
    for (int i = threadIdx.x; i < 256; i += blockDim.x) s_lut[i] = o.lut[i];
    if (threadIdx.x == 0) s_n = 0;
    __syncthreads();
    const int plen = (int)(qv.off[q + 1] - qv.off[q]);
    long long verified = 0;
    for (int i = threadIdx.x; i < ns; i += blockDim.x) {
        const Cand c = g[i];
        bool keep = false;
        uint64_t key = 0;
        if (c.pos < 0) {
            keep = true;
            key = c.val;
        } else {
            const int32_t s0 = o.soff[c.pos];
            const int tl = o.soff[c.pos + 1] - s0;
            verified++;
            const int d = dev::myers_any(s_peq, plen, o.chars + s0, tl, cut, s_lut);
            if (d <= cut) {
                keep = true;
                key = ((uint64_t)(uint32_t)d << 32) | a.ids[c.pos];
            }
        }
        if (keep) {
            const int slot = atomicAdd(&s_n, 1);
            keys[slot] = key;
        }
    }
    __syncthreads();
    if (verified) atomicAdd(&a.counters[CNT_VERIFIED], (unsigned long long)verified);
    const int nk = s_n;
    sort_and_emit(keys, nk, cap, k, a.out_keys + seg0, a.out_count + q);
}

void verify_edit(const VerifyArgs &a, const EditView &o, const QueryEdit &qv, hipStream_t st)
{
    if (a.nq == 0) return;
    hipLaunchKernelGGL(k_verify_edit, dim3((unsigned)((a.nq + 7) / 8 * 8)), dim3(256), 0, st, a, o, qv);
    check_launch(__func__);
}

// ---------------------------------------------------------------------------
// CSR assembly.
// ---------------------------------------------------------------------------
__global__ void k_csr_write(const uint64_t *__restrict__ out_keys, const int64_t *__restrict__ qoff,
                            const uint32_t *__restrict__ out_count, const int64_t *__restrict__ res_off, int64_t nq,
                            int is_edit, int64_t *__restrict__ ids, float *__restrict__ dist_f,
                            int32_t *__restrict__ dist_i)
{
    const int64_t q = blockIdx.x;
    if (q >= nq) return;
    const uint32_t cnt = out_count[q];
    const int64_t src = qoff[q], dst = res_off[q];
    for (uint32_t j = threadIdx.x; j < cnt; j += blockDim.x) {
        const uint64_t key = out_keys[src + j];
        ids[dst + j] = (int64_t)(uint32_t)key;
        const uint32_t hi = (uint32_t)(key >> 32);
        if (is_edit) dist_i[dst + j] = (int32_t)hi;
        else dist_f[dst + j] = __uint_as_float(hi);
    }
}

void csr_write(const uint64_t *out_keys, const int64_t *qoff, const uint32_t *out_count, const int64_t *res_off,
               int64_t nq, int is_edit, int64_t *ids, float *dist_f, int32_t *dist_i, hipStream_t st)
{
    if (nq == 0) return;
    hipLaunchKernelGGL(k_csr_write, dim3((unsigned)nq), dim3(64), 0, st, out_keys, qoff, out_count, res_off, nq,
                       is_edit, ids, dist_f, dist_i);
    check_launch(__func__);
}

}  // namespace k
}  // namespace gts
