// Candidate grouping by query, exact verification with per-query selection
// and (distance, id) ordering, and CSR assembly.
#include "dev_common.h"
#include "gts_internal.h"
#include "kernels.h"

namespace gts {
namespace k {


// Runs of equal query among a wave's 64 consecutive candidates (the sweep
// writes each lane's hits of one tile next to each other): the first lane of
// a run makes one atomic for the whole run.  Invalid lanes (the tail of the
// list, candidates left out by their query's epoch) may sit anywhere and end
// a run.  *head_lane = first lane of this lane's run; returns the run length
// at its first lane, 0 elsewhere.
__device__ __forceinline__ int query_run(int32_t q, bool valid, int *head_lane)
{
    const int lane = dev::lane_id();
    const int32_t prev = __shfl_up(q, 1, 64);
    const bool head = valid && (lane == 0 || prev != q);
    // both ballots by the whole wave, before any lane leaves
    const uint64_t hm = dev::ballot(head);
    const uint64_t stop = hm | ~dev::ballot(valid);           // a run ends before either
    const uint64_t upto = lane == 63 ? ~0ull : ((2ull << lane) - 1ull);
    *head_lane = (hm & upto) ? 63 - __clzll((long long)(hm & upto)) : lane;
    if (!head) return 0;
    const uint64_t after = stop & ~upto;
    const int end = after ? __ffsll((long long)after) - 1 : 64;
    return end - lane;
}

// Ascending bitonic sort of one 64-bit key per lane across the wave.
__device__ __forceinline__ uint64_t wave_sort64(uint64_t key)
{
    const int lane = dev::lane_id();
#pragma unroll
    for (int size = 2; size <= 64; size <<= 1)
#pragma unroll
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            const uint64_t other = __shfl_xor(key, stride, 64);
            const bool take_min = ((lane & size) == 0) == ((lane & stride) == 0);
            key = take_min ? (other < key ? other : key) : (other > key ? other : key);
        }
    return key;
}

// Number of runs of equal queries among the wave's 64 lanes.
__device__ __forceinline__ int query_runs(int32_t q)
{
    const int32_t prev = __shfl_up(q, 1, 64);
    return __popcll(dev::ballot(dev::lane_id() == 0 || prev != q));
}

// Grouping by query: a wave whose 64 candidates hold many runs sorts them by
// query first (invalid lanes, query -1, last), so every query of the window
// counts once however the producer interleaved them; the order inside a
// query's group is free (verification sorts by (distance, id)).
constexpr int kSortRuns = 16;
// Admission epochs (qep non-null): a tree candidate is dropped when its
// position was deleted at or before its query's epoch (del_ep[pos] <=
// qep[q]); the producers ran on the tombstones of the batch's earliest epoch.
__device__ __forceinline__ bool gone_at(const Cand &c, const uint32_t *del_ep, const uint32_t *qep)
{
    return qep != nullptr && c.q >= 0 && c.pos >= 0 && del_ep[c.pos] <= qep[c.q];
}

__global__ __launch_bounds__(256) void k_group_hist(const Cand *__restrict__ c, const CandCount *__restrict__ count,
                                                    int64_t cap, uint32_t *__restrict__ qcount,
                                                    const uint32_t *__restrict__ del_ep,
                                                    const uint32_t *__restrict__ qep)
{
    int64_t n = (int64_t)(*count > (CandCount)cap ? (CandCount)cap : *count);
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t b0 = (int64_t)blockIdx.x * blockDim.x + (threadIdx.x & ~63u); b0 < n; b0 += stride) {
        const int64_t i = b0 + dev::lane_id();
        int32_t q0 = -1;
        if (i < n) {
            if (qep) {
                const Cand ci = c[i];
                q0 = gone_at(ci, del_ep, qep) ? -1 : ci.q;
            } else {
                q0 = c[i].q;
            }
        }
        const int32_t q = query_runs(q0) > kSortRuns
                              ? (int32_t)(uint32_t)(wave_sort64((uint64_t)(uint32_t)q0 << 32) >> 32)
                              : q0;
        const bool valid = q != -1;
        int hl;
        const int len = query_run(q, valid, &hl);
        if (len) atomicAdd(&qcount[q], (uint32_t)len);
    }
}

void group_hist(const Cand *c, const CandCount *count, int64_t cap, uint32_t *qcount, const uint32_t *del_ep,
                const uint32_t *qep, hipStream_t st)
{
    hipLaunchKernelGGL(k_group_hist, dim3(2048), dim3(256), 0, st, c, count, cap, qcount, del_ep, qep);
    check_launch(__func__);
}

// Exclusive scan of n counts into out[0..n], one workgroup of 1024 threads.
__global__ __launch_bounds__(1024) void k_scan_u32(const uint32_t *__restrict__ in, int64_t n,
                                                   int64_t *__restrict__ out)
{
    // one workgroup, tiles of 4096 entries (4 consecutive per thread): wave
    // scans of the per-thread sums, then of the 16 wave totals, plus the
    // running total of the earlier tiles
    __shared__ int64_t s_w[16];
    __shared__ int64_t s_carry;
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    if (t == 0) s_carry = 0;
    __syncthreads();
    for (int64_t base = 0; base < n; base += 4096) {
        int64_t v[4], sum = 0;
#pragma unroll
        for (int u = 0; u < 4; u++) {
            const int64_t i = base + 4 * t + u;
            v[u] = i < n ? (int64_t)in[i] : 0;
            sum += v[u];
        }
        int64_t x = sum;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int64_t y = __shfl_up(x, o, 64);
            if (lane >= o) x += y;
        }
        if (lane == 63) s_w[wv] = x;
        __syncthreads();
        if (wv == 0) {
            int64_t w = lane < 16 ? s_w[lane] : 0;
#pragma unroll
            for (int o = 1; o < 16; o <<= 1) {
                const int64_t y = __shfl_up(w, o, 64);
                if (lane >= o) w += y;
            }
            if (lane < 16) s_w[lane] = w;
        }
        __syncthreads();
        int64_t run = s_carry + (wv ? s_w[wv - 1] : 0) + x - sum;
#pragma unroll
        for (int u = 0; u < 4; u++) {
            const int64_t i = base + 4 * t + u;
            if (i < n) out[i] = run;
            run += v[u];
        }
        __syncthreads();
        if (t == 1023) s_carry = run;
        __syncthreads();
    }
    if (t == 0) out[n] = s_carry;
}

void scan_u32(const uint32_t *in, int64_t n, int64_t *out, hipStream_t st)
{
    hipLaunchKernelGGL(k_scan_u32, dim3(1), dim3(1024), 0, st, in, n, out);
    check_launch(__func__);
}

__global__ __launch_bounds__(256) void k_group_scatter(const Cand *__restrict__ c, const CandCount *__restrict__ count,
                                                       int64_t cap, const int64_t *__restrict__ qoff,
                                                       uint32_t *__restrict__ cursor, Cand *__restrict__ grouped,
                                                       int64_t grouped_cap, const uint32_t *__restrict__ del_ep,
                                                       const uint32_t *__restrict__ qep)
{
    int64_t n = (int64_t)(*count > (CandCount)cap ? (CandCount)cap : *count);
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int lane = dev::lane_id();
    for (int64_t b0 = (int64_t)blockIdx.x * blockDim.x + (threadIdx.x & ~63u); b0 < n; b0 += stride) {
        const int64_t i = b0 + lane;
        Cand c0;
        c0.q = -1;
        c0.pos = 0;
        c0.val = 0;
        if (i < n) c0 = c[i];
        if (gone_at(c0, del_ep, qep)) c0.q = -1;
        // sort the wave's candidates by query, then take each record from
        // the lane that loaded it
        Cand cd = c0;
        if (query_runs(c0.q) > kSortRuns) {   // wave-uniform
            const uint64_t key = wave_sort64(((uint64_t)(uint32_t)c0.q << 32) | (uint32_t)lane);
            const int src = (int)(key & 63u);
            cd.q = (int32_t)(uint32_t)(key >> 32);
            cd.pos = __shfl(c0.pos, src, 64);
            cd.val = __shfl(c0.val, src, 64);
        }
        const bool valid = cd.q != -1;
        int hl;
        const int len = query_run(cd.q, valid, &hl);
        uint32_t base = 0;
        if (len) base = atomicAdd(&cursor[cd.q], (uint32_t)len);
        base = __shfl(base, hl, 64);
        const int64_t dst = valid ? qoff[cd.q] + base + (uint32_t)(lane - hl) : grouped_cap;
        if (dst < grouped_cap) grouped[dst] = cd;
    }
}

void group_scatter(const Cand *c, const CandCount *count, int64_t cap, const int64_t *qoff, uint32_t *cursor,
                   Cand *grouped, int64_t grouped_cap, const uint32_t *del_ep, const uint32_t *qep, hipStream_t st)
{
    hipLaunchKernelGGL(k_group_scatter, dim3(2048), dim3(256), 0, st, c, count, cap, qoff, cursor, grouped,
                       grouped_cap, del_ep, qep);
    check_launch(__func__);
}

// Sort the keys of one query (in LDS or, for a large segment, in its
// power-of-two scratch run) and write the first `keep` to out.

// ---------------------------------------------------------------------------
// L2: per query, one workgroup.  kNN queries first keep only candidates
// whose distance interval can reach the k smallest upper bounds: from the
// bf16 estimate e of d^2, d lies in [sqrt(e - eps) - eq - ex,
// sqrt(e + eps) + eq + ex].  Then each kept candidate gets its exact float32
// distance (direct difference, 16 lanes per candidate); range queries keep
// d <= r, kNN queries keep everything; keys are sorted by (d, id).
// ---------------------------------------------------------------------------
__device__ __forceinline__ void l2_interval(const Cand &c, float qnn, float qerr, const L2View &o, float eps_a,
                                            float eps_b, float eps_c, float delta, float *lo, float *hi,
                                            bool angular = false)
{
    if (c.pos < 0 && angular) {
        // a cache entry's key holds its angle, not d: no interval (always kept,
        // never tightens the bound; the k-th upper end of the others still
        // bounds the k-th distance)
        *lo = 0.f;
        *hi = INFINITY;
        return;
    }
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

// Exact float32 rechecks of the candidates [i0, i1) of query q by one wave.
// The candidates stream in steps of 64 (one per lane), the next step loading
// while the current one is decided: cache entries, whose distance is already
// known, are kept at once; a kNN candidate whose lower interval end exceeds
// the bound ub is dropped; the positions that need a recheck go through a
// ring of 128 entries in LDS, and every kBatch of them make a batch: 16 lanes
// per candidate, kBatch / 4 candidates per 16-lane group, rows and ids all
// requested before any is used, the same strided float32 sum as every other
// exact L2 distance here (the query slice in registers when the row has at
// most 128 floats).  emit(keep, key) takes every lane's decision and is
// called by the whole wave.
constexpr int kWaveSteps = kVerifyBlockMin / 64;   // 64-candidate steps of a wave-mode query
static_assert(kVerifyBlockMin <= kWaveSortCap, "a wave verifies at most its LDS run");
constexpr int kRing = 128;
constexpr int kBatch = 24;                   // rechecks in flight per wave (six per 16-lane group)
static_assert(kBatch % 4 == 0 && kBatch + 64 <= kRing, "recheck batch");

struct RecheckCtx {
    const float *qrow;
    float qr[8];
    float qnn, qerr, base, ub;
    int k;
    bool sel;                                // ub in force (kNN)
    bool est;                                // candidates carry bf16 estimates
};

template <bool kShort, bool kCheck, bool kL1, class Emit>
__device__ __forceinline__ void recheck_chunk(const VerifyArgs &a, const L2View &o, const RecheckCtx &rc,
                                              float delta, float eps_a, float eps_b, float eps_c, const Cand *g,
                                              int i0, int i1, int32_t *ring, long long *verified, long long *viol,
                                              Emit &emit)
{
    // ring[0, kRing): positions; ring[kRing, 2 kRing): their bf16 estimates
    uint32_t *ring_est = reinterpret_cast<uint32_t *>(ring + kRing);
    const int lane = threadIdx.x & 63, grp = lane >> 4, sl = lane & 15;
    const int nu = (i1 - i0 + 63) >> 6;
    int head = 0, tail = 0;                      // ring cursors (wave-uniform)
    auto batch = [&](int cnt) __attribute__((always_inline)) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        constexpr int U = kBatch / 4;
        int32_t p[U];
        uint32_t ev[U];
        bool nd[U];
#pragma unroll
        for (int uu = 0; uu < U; uu++) {
            const int j = 4 * uu + grp;
            nd[uu] = j < cnt;
            p[uu] = nd[uu] ? ring[(head + j) & (kRing - 1)] : 0;
            ev[uu] = kCheck && nd[uu] && sl == 0 ? ring_est[(head + j) & (kRing - 1)] : 0u;
        }
        uint32_t idv[U];
        float acc[U];
#pragma unroll
        for (int uu = 0; uu < U; uu++) idv[uu] = nd[uu] && sl == 0 ? a.ids[p[uu]] : 0u;
        if (kShort) {
            float xv[U][8];
#pragma unroll
            for (int uu = 0; uu < U; uu++) {
                const float *x = o.X32 + (size_t)p[uu] * o.dp;
#pragma unroll
                for (int t = 0; t < 8; t++) xv[uu][t] = nd[uu] && sl + 16 * t < o.dp ? x[sl + 16 * t] : 0.f;
            }
            // coordinates beyond dp are zero on both sides: fmaf(0, 0, acc) == acc
#pragma unroll
            for (int uu = 0; uu < U; uu++) {
                acc[uu] = 0.f;
#pragma unroll
                for (int t = 0; t < 8; t++) acc[uu] = dev::dterm<kL1>(acc[uu], rc.qr[t], xv[uu][t]);
            }
        } else {
            const float *x[U];
#pragma unroll
            for (int uu = 0; uu < U; uu++) {
                acc[uu] = 0.f;
                x[uu] = nd[uu] ? o.X32 + (size_t)p[uu] * o.dp : rc.qrow;
            }
            for (int d = sl; d < o.dp; d += 16) {
                const float qd = rc.qrow[d];
#pragma unroll
                for (int uu = 0; uu < U; uu++) acc[uu] = dev::dterm<kL1>(acc[uu], qd, x[uu][d]);
            }
        }
#pragma unroll
        for (int uu = 0; uu < U; uu++)
#pragma unroll
            for (int off = 8; off > 0; off >>= 1) acc[uu] += __shfl_xor(acc[uu], off, 16);
#pragma unroll
        for (int uu = 0; uu < U; uu++) {
            const bool mine = nd[uu] && sl == 0;
            const float d = dev::dfinish<kL1>(acc[uu]);
            if (mine) (*verified)++;
            if (kCheck && mine && rc.est) {
                // invariant of the bf16 selection: the exact distance lies in
                // the candidate's interval (up to the float32 error of d)
                Cand c;
                c.q = 0;
                c.pos = p[uu];
                c.val = ev[uu];
                float lo, hi;
                l2_interval(c, rc.qnn, rc.qerr, o, eps_a, eps_b, eps_c, delta, &lo, &hi, a.angular != 0);
                if (d < lo * (1.f - 2.f * delta) || d > hi * (1.f + 2.f * delta)) (*viol)++;
            }
            emit(mine && (rc.k > 0 || d <= rc.base),
                 ((uint64_t)__float_as_uint(dev::out_dist(d, a.angular != 0)) << 32) | idv[uu]);
        }
    };
    // one 64-candidate step at a time, the next step's candidates loading
    // while this one is staged and its full batches run
    auto load = [&](int u, Cand *c) __attribute__((always_inline)) {
        const int i = i0 + lane + 64 * u;
        c->q = 0;
        c->pos = -1;
        c->val = 0;
        if (i < i1) *c = g[i];
        return i < i1;
    };
    Cand cn;
    bool vn = load(0, &cn);
    for (int u = 0; u < nu; u++) {
        const Cand c = cn;
        const bool v = vn;
        if (u + 1 < nu) vn = load(u + 1, &cn);
        bool need = v && c.pos >= 0;
        if (need && rc.sel && rc.ub < INFINITY) {
            float lo, hi;
            l2_interval(c, rc.qnn, rc.qerr, o, eps_a, eps_b, eps_c, delta, &lo, &hi, a.angular != 0);
            need = lo <= rc.ub;
        }
        emit(v && c.pos < 0, c.val);                 // known distance (cache list)
        const uint64_t m = dev::ballot(need);
        if (need) {
            ring[(tail + dev::lanes_below(m)) & (kRing - 1)] = c.pos;
            if (kCheck) ring_est[(tail + dev::lanes_below(m)) & (kRing - 1)] = (uint32_t)c.val;
        }
        tail += __popcll(m);
        while (tail - head >= kBatch) {
            batch(kBatch);
            head += kBatch;
        }
    }
    if (tail > head) batch(tail - head);
}

// One workgroup for query q (more candidates than one wave takes).  kNN:
// the k-th smallest upper interval end, found by a 32-step binary search
// over the float bits with block-wide counts of the values held in LDS,
// bounds the answer set (when the candidates fit the LDS run).  Each wave
// rechecks an equal share of whole 64-candidate steps; kept keys are compacted
// per wave (one LDS atomic reserves the wave's slots) and sorted in LDS
// (s_keys, kSortCapL2) or in the query's scratch run.
template <bool kShort, bool kCheck, bool kL1>
__device__ void verify_l2_block(const VerifyArgs &a, const L2View &o, const QueryL2 &qv, float delta, float eps_a,
                                float eps_b, float eps_c, int64_t q, uint64_t *s_keys, int32_t *ring, bool est)
{
    __shared__ int s_n;
    const int64_t seg0 = a.qoff[q];
    const int ns = (int)(a.qoff[q + 1] - seg0);
    const int k = a.kq ? a.kq[q] : 0;
    const int64_t boff = a.big_off ? a.big_off[q] : -1;
    const bool big = boff >= 0;
    uint64_t *keys = big ? a.scratch + boff : s_keys;
    const int64_t cap = big ? dev::next_pow2(ns) : kSortCapL2;
    const Cand *g = a.grouped + seg0;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    RecheckCtx rc;
    rc.qrow = qv.Q32 + (size_t)q * o.dp;
    rc.qnn = qv.qn[q];
    rc.qerr = qv.qe[q];
    rc.base = a.base[q];
    rc.k = k;
    rc.ub = INFINITY;
    rc.est = est;
    rc.sel = est && k > 0 && ns > k && !big;
    if (threadIdx.x == 0) s_n = 0;
    if (rc.sel) {
        for (int i = threadIdx.x; i < ns; i += blockDim.x) {
            float lo, hi;
            l2_interval(g[i], rc.qnn, rc.qerr, o, eps_a, eps_b, eps_c, delta, &lo, &hi, a.angular != 0);
            s_keys[i] = (uint64_t)__float_as_uint(hi);
        }
        // the k-th smallest hi (hi >= 0: float order = bit order) by a radix
        // select, 8-bit digits from the top: per round a 256-bin LDS
        // histogram of the keys matching the digits chosen so far, then wave
        // 0 finds the digit holding the k-th
        __shared__ uint32_t s_hist[256];
        __shared__ uint32_t s_pick[2];
        uint32_t prefix = 0u, pmask = 0u, kk = (uint32_t)k;
        for (int shift = 24; shift >= 0; shift -= 8) {
            for (int i = threadIdx.x; i < 256; i += blockDim.x) s_hist[i] = 0u;
            __syncthreads();
            for (int i = threadIdx.x; i < ns; i += blockDim.x) {
                const uint32_t v = (uint32_t)s_keys[i];
                if ((v & pmask) == prefix) atomicAdd(&s_hist[(v >> shift) & 255u], 1u);
            }
            __syncthreads();
            if (wave == 0) {
                uint32_t c[4];
                int sum = 0;
#pragma unroll
                for (int u = 0; u < 4; u++) {
                    c[u] = s_hist[4 * lane + u];
                    sum += (int)c[u];
                }
                int total;
                uint32_t before = (uint32_t)dev::wave_excl_scan(sum, &total);
                if (before < kk && kk <= before + (uint32_t)sum) {
                    int u = 0;
                    while (before + c[u] < kk) before += c[u++];
                    s_pick[0] = (uint32_t)(4 * lane + u);
                    s_pick[1] = kk - before;
                }
            }
            __syncthreads();
            prefix |= s_pick[0] << shift;
            pmask |= 255u << shift;
            kk = s_pick[1];
            __syncthreads();
        }
        rc.ub = __uint_as_float(prefix) * (1.f + 4.f * delta);
    }
    __syncthreads();
    const int sl = lane & 15;
    if (kShort) {
#pragma unroll
        for (int t = 0; t < 8; t++) rc.qr[t] = sl + 16 * t < o.dp ? rc.qrow[sl + 16 * t] : 0.f;
    }
    long long verified = 0, viol = 0;
    auto emit = [&](bool keep, uint64_t key) __attribute__((always_inline)) {
        const uint64_t m = dev::ballot(keep);
        if (m) {
            int slot0 = 0;
            if (lane == 0) slot0 = atomicAdd(&s_n, __popcll(m));
            slot0 = __shfl(slot0, 0, 64);
            if (keep) keys[slot0 + dev::lanes_below(m)] = key;
        }
    };
    // the candidates split evenly over the waves (whole 64-candidate steps)
    const int nw = (int)(blockDim.x >> 6);
    const int steps = (ns + 63) >> 6, per = (steps + nw - 1) / nw;
    const int c0 = min(ns, 64 * per * wave), c1 = min(ns, 64 * per * (wave + 1));
    if (c0 < c1)
        recheck_chunk<kShort, kCheck, kL1>(a, o, rc, delta, eps_a, eps_b, eps_c, g, c0, c1, ring, &verified, &viol,
                                           emit);
    __syncthreads();
    for (int o2 = 32; o2 > 0; o2 >>= 1) verified += __shfl_xor(verified, o2, 64);
    for (int o2 = 32; o2 > 0; o2 >>= 1) viol += __shfl_xor(viol, o2, 64);
    if (lane == 0 && verified) count_add(a.counters, CNT_VERIFIED, (unsigned long long)verified);
    if (lane == 0 && viol) count_add(a.counters, CNT_BOUND_VIOL, (unsigned long long)viol);
    const int nk = s_n;
    dev::sort_and_emit(keys, nk, cap, k, a.out_keys + seg0, a.out_count + q);
}


// One wave for query q (at most kVerifyBlockMin candidates).  kNN: the k-th
// smallest upper interval end over the candidates, found by a 32-step
// binary search over the float bits (counting with ballots over the values
// each lane holds in registers), bounds the answer set; then one chunk of
// rechecks (above).  Kept keys are compacted with ballots into the wave's
// LDS run and sorted there.
template <bool kShort, bool kCheck, bool kL1>
__device__ void verify_l2_wave(const VerifyArgs &a, const L2View &o, const QueryL2 &qv, float delta, float eps_a,
                               float eps_b, float eps_c, int64_t q, uint64_t *keys, int32_t *ring, bool est)
{
    const int lane = threadIdx.x & 63;
    const int64_t seg0 = a.qoff[q];
    const int ns = (int)(a.qoff[q + 1] - seg0);
    const int k = a.kq ? a.kq[q] : 0;
    const Cand *g = a.grouped + seg0;
    RecheckCtx rc;
    rc.qrow = qv.Q32 + (size_t)q * o.dp;
    rc.qnn = qv.qn[q];
    rc.qerr = qv.qe[q];
    rc.base = a.base[q];
    rc.k = k;
    rc.ub = INFINITY;
    rc.est = est;
    rc.sel = est && k > 0 && ns > k;
    if (rc.sel) {
        uint32_t hv[kWaveSteps];
#pragma unroll
        for (int u = 0; u < kWaveSteps; u++) {
            const int i = lane + 64 * u;
            hv[u] = 0xffffffffu;
            if (i < ns) {
                float lo, hi;
                l2_interval(g[i], rc.qnn, rc.qerr, o, eps_a, eps_b, eps_c, delta, &lo, &hi, a.angular != 0);
                hv[u] = __float_as_uint(hi);
            }
        }
        // smallest v with #{hi <= v} >= k (hi >= 0, so float order = bit order;
        // the padding 0xffffffff is never counted: mid < 0xffffffff)
        const int nu = (ns + 63) >> 6;
        uint32_t lo_v = 0u, hi_v = 0xffffffffu;
        while (lo_v < hi_v) {
            const uint32_t mid = lo_v + ((hi_v - lo_v) >> 1);
            int c = 0;
#pragma unroll
            for (int u = 0; u < kWaveSteps; u++)
                if (u < nu) c += __popcll(dev::ballot(hv[u] <= mid));
            if (c >= k) hi_v = mid;
            else lo_v = mid + 1u;
        }
        rc.ub = __uint_as_float(lo_v) * (1.f + 4.f * delta);
    }
    const int sl = lane & 15;
    if (kShort) {
#pragma unroll
        for (int t = 0; t < 8; t++) rc.qr[t] = sl + 16 * t < o.dp ? rc.qrow[sl + 16 * t] : 0.f;
    }
    long long verified = 0, viol = 0;
    int nk = 0;
    auto emit = [&](bool keep, uint64_t key) __attribute__((always_inline)) {
        const uint64_t m = dev::ballot(keep);
        if (keep) keys[nk + dev::lanes_below(m)] = key;
        nk += __popcll(m);
    };
    recheck_chunk<kShort, kCheck, kL1>(a, o, rc, delta, eps_a, eps_b, eps_c, g, 0, ns, ring, &verified, &viol, emit);
    for (int o2 = 32; o2 > 0; o2 >>= 1) verified += __shfl_xor(verified, o2, 64);
    for (int o2 = 32; o2 > 0; o2 >>= 1) viol += __shfl_xor(viol, o2, 64);
    if (lane == 0 && verified) count_add(a.counters, CNT_VERIFIED, (unsigned long long)verified);
    if (lane == 0 && viol) count_add(a.counters, CNT_BOUND_VIOL, (unsigned long long)viol);
    const int P = dev::next_pow2(nk > 1 ? nk : 1);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    for (int i = nk + lane; i < P; i += 64) keys[i] = ~0ull;
    dev::wave_bitonic_sort(keys, P);
    const int nout = (k > 0 && k < nk) ? k : nk;
    for (int j = lane; j < nout; j += 64) a.out_keys[seg0 + j] = keys[j];
    if (lane == 0) a.out_count[q] = (uint32_t)nout;
}

// One persistent launch for both forms.  First the queries of the order's
// head (more than kVerifyBlockMin candidates), a whole workgroup each, dealt
// to the workgroups in turn.  Then each wave takes the rest on its own from
// a work queue, one query per grab, so a wave that finishes early goes on
// at once (a workgroup's LDS is held until its last wave ends) and the
// longest queries, which come first, start first.  The queue is split over
// the XCDs (runs of kVerifyRun consecutive queries dealt to the nx =
// min(8, workgroups) queues in turn, workgroup b serving queue b mod nx;
// workgroups are dealt to the XCDs round robin), each cursor on its own
// 128-byte line: a single cursor taken by every wave of the chip serialised
// the grabs.
// Every grab is made without lane-divergent control flow (all lanes issue
// the atomic, lane 0 adding 1; the chunk is lane 0's value in a scalar
// register), so the exit test is a scalar branch of the whole wave.
template <bool kShort, bool kCheck, bool kL1>
__global__ __launch_bounds__(256, 4) void k_verify_l2(VerifyArgs a, L2View o, QueryL2 qv, float delta, float eps_a,
                                                      float eps_b, float eps_c, const int32_t *__restrict__ order,
                                                      int n_blk_arg, const int32_t *__restrict__ n_blk_dev,
                                                      uint32_t *__restrict__ ctr, int est)
{
    __shared__ uint64_t s_mem[kSortCapL2];
    __shared__ int32_t s_ring[4][2 * kRing];
    static_assert(4 * kWaveSortCap <= kSortCapL2, "wave runs must fit the workgroup's LDS");
    const int n_blk = __builtin_amdgcn_readfirstlane(n_blk_dev ? *n_blk_dev : n_blk_arg);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int it = blockIdx.x; it < n_blk; it += gridDim.x) {
        verify_l2_block<kShort, kCheck, kL1>(a, o, qv, delta, eps_a, eps_b, eps_c, order[it], s_mem, s_ring[wave],
                                             est != 0);
        __syncthreads();
    }
    const int n_wave = (int)a.nq - n_blk;
    const int nx = gridDim.x < 8 ? (int)gridDim.x : 8;
    const int x = (int)(blockIdx.x % nx);
    uint32_t *cur = ctr + x * kVerifyCursorStride;
    for (;;) {
        const uint32_t got = atomicAdd(cur, lane == 0 ? 1u : 0u);
        const int64_t j = __builtin_amdgcn_readfirstlane((int)got);
        // this queue's j-th query: runs of kVerifyRun consecutive queries of
        // the order belong to one queue (neighbours share candidate rows in
        // the XCD's L2), the runs dealt to the queues in turn
        const int64_t it = ((j / kVerifyRun) * nx + x) * kVerifyRun + j % kVerifyRun;
        if (it >= n_wave) break;
        // the wave's LDS run and ring are reused: the last query's reads
        // come before this one's writes
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        verify_l2_wave<kShort, kCheck, kL1>(a, o, qv, delta, eps_a, eps_b, eps_c, order[n_blk + it],
                                            s_mem + wave * kWaveSortCap, s_ring[wave], est != 0);
    }
}

void verify_l2(const VerifyArgs &a, const L2View &o, const QueryL2 &qv, float delta, const int32_t *order, int n_blk,
               bool est, bool check, hipStream_t st, bool l1, const int32_t *n_blk_dev, uint32_t *ctr)
{
    if (a.nq == 0) return;
    const float u = 5.9604645e-8f;
    const int D = o.ksteps * 32;
    const float eps_a = 2.f * (D + 8) * u, eps_b = 2.f * (4 * D + 8) * u, eps_c = 8.f * u;
    // persistent: four workgroups per CU (the LDS holds four), fewer for a
    // small batch
    int dev = 0, cus = 256;
    GTS_HIP(hipGetDevice(&dev));
    GTS_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    const unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>(4 * (int64_t)cus, (a.nq + 3) / 4));
#define VL(S, C, M)                                                                                           \
    hipLaunchKernelGGL((k_verify_l2<S, C, M>), dim3(grid), dim3(256), 0, st, a, o, qv, delta, eps_a, eps_b, eps_c, \
                       order, n_blk, n_blk_dev, ctr, est ? 1 : 0)
    const bool chk = check && est;
    if (l1) {
        // Manhattan: no bf16 estimates, every candidate takes its float32 distance
        require(!est, "verify_l2: the L1 metric has no bf16 selection");
        if (o.dp <= 128) VL(true, false, true);
        else VL(false, false, true);
    } else if (o.dp <= 128) {
        if (chk) VL(true, true, false);
        else VL(true, false, false);
    } else {
        if (chk) VL(false, true, false);
        else VL(false, false, false);
    }
#undef VL
    check_launch(__func__);
}

// ---------------------------------------------------------------------------
// EDIT: per query, one workgroup; the query's match table sits in LDS and
// every lane verifies one candidate (object string as the text) with the
// early-exit cutoff floor(base); kept keys are sorted by (d, id).  kBand:
// every cutoff of the launch is at most 63, so only the banded one-word
// recurrence is compiled in (fewer registers, more waves in flight).
// ---------------------------------------------------------------------------
template <bool kBand>
__global__ __launch_bounds__(256) void k_verify_edit(VerifyArgs a, EditView o, QueryEdit qv)
{
    __shared__ uint64_t s_keys[kSortCap];
    __shared__ uint64_t s_peq[257 * 4];
    __shared__ uint8_t s_lut[256];
    __shared__ int s_n;
    // one query per workgroup in batch order: the Myers work per query varies
    // a lot, and interleaving the queries over the XCDs balances it
    const int64_t q = blockIdx.x;
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
            const int d = kBand ? dev::myers_banded(s_peq, 4, plen, o.chars + s0, tl, cut, s_lut)
                                : dev::myers_any(s_peq, plen, o.chars + s0, tl, cut, s_lut);
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
    if (verified) count_add(a.counters, CNT_VERIFIED, (unsigned long long)verified);
    const int nk = s_n;
    dev::sort_and_emit(keys, nk, cap, k, a.out_keys + seg0, a.out_count + q);
}

void verify_edit(const VerifyArgs &a, const EditView &o, const QueryEdit &qv, bool band_only, hipStream_t st)
{
    if (a.nq == 0) return;
    if (band_only) hipLaunchKernelGGL(k_verify_edit<true>, dim3((unsigned)a.nq), dim3(256), 0, st, a, o, qv);
    else hipLaunchKernelGGL(k_verify_edit<false>, dim3((unsigned)a.nq), dim3(256), 0, st, a, o, qv);
    check_launch(__func__);
}

// ---------------------------------------------------------------------------
// Verification plan on the device (graph-replayed searches, which read no
// counts on the host): per query its candidate count from the grouping
// offsets; queries beyond the LDS sort get a power-of-two run of the scratch
// (offsets by a scan); the verification order lists the queries by
// verify_class (class sizes counted with atomics, then each query placed at
// its class's base plus an atomic cursor: the order inside a class varies
// from run to run, the answers do not).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_verify_need(const int64_t *__restrict__ qoff, int64_t ng, int64_t sort_cap,
                                                     uint32_t *__restrict__ need, uint32_t *__restrict__ cls)
{
    // class counts and the largest count aggregated per wave (one atomic per
    // class per wave: 20,000 queries on a handful of words serialised)
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int lane = threadIdx.x & 63;
    const bool valid = q < ng;
    const int64_t ns = valid ? qoff[q + 1] - qoff[q] : 0;
    if (valid) {
        uint32_t p = 0;
        if (ns > sort_cap) {
            p = 1;
            while ((int64_t)p < ns) p <<= 1;
        }
        need[q] = p;
    }
    const int c = valid ? verify_class(ns) : -1;
#pragma unroll
    for (int j = 0; j < kVerifyClasses; j++) {
        const uint64_t m = dev::ballot(c == j);
        if (lane == 0 && m) atomicAdd(&cls[j], (uint32_t)__popcll(m));   // (result unused)
    }
    uint32_t mx = (uint32_t)ns;
    for (int o = 32; o > 0; o >>= 1) mx = max(mx, (uint32_t)__shfl_xor((int)mx, o, 64));
    if (lane == 0 && mx) atomicMax(&cls[2 * kVerifyClasses], mx);
}

__global__ __launch_bounds__(256) void k_verify_lists(const int64_t *__restrict__ qoff, const uint32_t *__restrict__ need,
                                                      const int64_t *__restrict__ need_off, uint32_t *__restrict__ cls,
                                                      int64_t ng, int64_t *__restrict__ big_off,
                                                      int32_t *__restrict__ order, int32_t *__restrict__ n_blk)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int lane = threadIdx.x & 63;
    if (q == 0 && n_blk) *n_blk = (int32_t)cls[0];
    const bool valid = q < ng;
    if (valid) big_off[q] = need[q] ? need_off[q] : -1;
    const int c = valid ? verify_class(qoff[q + 1] - qoff[q]) : -1;
    // one cursor reservation per class per wave, each lane ranked among the
    // wave's lanes of its class
    const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    int32_t slot = -1;
#pragma unroll
    for (int j = 0; j < kVerifyClasses; j++) {
        const uint64_t m = dev::ballot(c == j);
        if (!m) continue;
        // (every lane issues the atomic, lane 0 with the count: no
        // lane-divergent control flow around the cross-lane read)
        uint32_t base = 0;
        for (int i = 0; i < j; i++) base += cls[i];
        const uint32_t got = atomicAdd(&cls[kVerifyClasses + j], lane == 0 ? (uint32_t)__popcll(m) : 0u);
        const uint32_t at = base + (uint32_t)__builtin_amdgcn_readfirstlane((int)got);
        if (c == j) slot = (int32_t)(at + (uint32_t)__popcll(m & below));
    }
    if (valid) order[slot] = (int32_t)q;
}

void verify_plan_count(const int64_t *qoff, int64_t ng, int64_t sort_cap, uint32_t *need, int64_t *need_off,
                       uint32_t *cls, hipStream_t st)
{
    const unsigned g = (unsigned)((ng + 256) / 256);
    fill_u32(cls, kVerifyPlanWords, 0u, st);
    hipLaunchKernelGGL(k_verify_need, dim3(g), dim3(256), 0, st, qoff, ng, sort_cap, need, cls);
    check_launch("verify_plan_count");
    scan_u32(need, ng, need_off, st);
}

void verify_plan_lists(const int64_t *qoff, int64_t ng, const uint32_t *need, const int64_t *need_off, uint32_t *cls,
                       int64_t *big_off, int32_t *order, int32_t *n_blk, hipStream_t st)
{
    const unsigned g = (unsigned)((ng + 256) / 256);
    hipLaunchKernelGGL(k_verify_lists, dim3(g), dim3(256), 0, st, qoff, need, need_off, cls, ng, big_off, order,
                       n_blk);
    check_launch("verify_plan_lists");
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

__global__ void k_perm_counts(const uint32_t *__restrict__ out_count, const int32_t *__restrict__ perm, int64_t nq,
                              uint32_t *__restrict__ cc)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nq) cc[perm ? perm[i] : i] = out_count[i];
}

void perm_counts(const uint32_t *out_count, const int32_t *perm, int64_t nq, uint32_t *cc, hipStream_t st)
{
    if (nq == 0) return;
    hipLaunchKernelGGL(k_perm_counts, dim3((unsigned)((nq + 255) / 256)), dim3(256), 0, st, out_count, perm, nq, cc);
    check_launch(__func__);
}

__global__ void k_emit_result(const uint64_t *__restrict__ out_keys, const int64_t *__restrict__ qoff,
                              const uint32_t *__restrict__ out_count, const int32_t *__restrict__ perm,
                              const int64_t *__restrict__ dst_off, int64_t nq, int is_edit, int64_t *__restrict__ ids,
                              float *__restrict__ dist_f, int32_t *__restrict__ dist_i, int64_t cap)
{
    const int64_t i = blockIdx.x;
    if (i >= nq) return;
    const int64_t src = qoff[i], dst = dst_off[perm ? perm[i] : i];
    // cap >= 0: only entries below the output capacity are written
    const uint32_t cnt = cap < 0 ? out_count[i] : (uint32_t)max<int64_t>(0, min<int64_t>(out_count[i], cap - dst));
    for (uint32_t j = threadIdx.x; j < cnt; j += blockDim.x) {
        const uint64_t key = out_keys[src + j];
        ids[dst + j] = (int64_t)(uint32_t)key;
        const uint32_t hi = (uint32_t)(key >> 32);
        if (is_edit) dist_i[dst + j] = (int32_t)hi;
        else dist_f[dst + j] = __uint_as_float(hi);
    }
}

void emit_result(const uint64_t *out_keys, const int64_t *qoff, const uint32_t *out_count, const int32_t *perm,
                 const int64_t *dst_off, int64_t nq, int is_edit, int64_t *ids, float *dist_f, int32_t *dist_i,
                 hipStream_t st, int64_t cap)
{
    if (nq == 0) return;
    hipLaunchKernelGGL(k_emit_result, dim3((unsigned)nq), dim3(64), 0, st, out_keys, qoff, out_count, perm, dst_off,
                       nq, is_edit, ids, dist_f, dist_i, cap);
    check_launch(__func__);
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
