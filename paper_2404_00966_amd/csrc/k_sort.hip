// Query order by home (leaf or cell) on the device: a stable least-
// significant-digit radix sort of the home keys carrying the query index,
// so the permutation is the same on every run and no host round trip sits
// between the search for the homes and the first kernel that reads the
// queries in the new order.
//
// Each pass sorts by one 8-bit digit in three launches over a fixed split of
// the input into contiguous ranges, one per workgroup:
//   k_digit_hist    : per range, the count of each digit value (LDS atomics),
//                     stored digit-major: hist[digit * ranges + range];
//   k_scan_u32      : exclusive scan of that table, so entry (d, r) is where
//                     range r's first element of digit d goes;
//   k_digit_scatter : per range, in input order, 1,024 elements at a time:
//                     inside a wave, the lanes holding the same digit are
//                     found with eight ballots (one per bit) and ranked by
//                     the lanes below; per-wave digit counts in LDS give the
//                     offsets of the waves before; a running per-digit base
//                     carries across the range's chunks.  Equal digits keep
//                     their input order, which makes the pass stable.
#include "dev_common.h"
#include "gts_internal.h"
#include "kernels.h"

namespace gts {
namespace k {

namespace {

constexpr int kRadix = 256;
constexpr int kSortThreads = 1024;          // 16 waves
constexpr int kSortWaves = kSortThreads / 64;
constexpr int64_t kRangeItems = 4096;       // elements per workgroup range

}  // namespace

__global__ void k_home_keys(const int32_t *__restrict__ home, int stride, int64_t nq, uint32_t *__restrict__ key,
                            int32_t *__restrict__ idx)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < nq) {
        key[q] = (uint32_t)home[q * stride];
        idx[q] = (int32_t)q;
    }
}

__global__ __launch_bounds__(kSortThreads) void k_digit_hist(const uint32_t *__restrict__ key, int64_t n, int shift,
                                                             int64_t ranges, uint32_t *__restrict__ hist)
{
    __shared__ uint32_t s_h[kRadix];
    for (int i = threadIdx.x; i < kRadix; i += blockDim.x) s_h[i] = 0u;
    __syncthreads();
    const int64_t r = blockIdx.x;
    const int64_t b = r * kRangeItems, e = min<int64_t>(n, b + kRangeItems);
    for (int64_t i = b + threadIdx.x; i < e; i += blockDim.x) atomicAdd(&s_h[(key[i] >> shift) & (kRadix - 1)], 1u);
    __syncthreads();
    for (int d = threadIdx.x; d < kRadix; d += blockDim.x) hist[(int64_t)d * ranges + r] = s_h[d];
}

__global__ __launch_bounds__(kSortThreads) void k_digit_scatter(const uint32_t *__restrict__ key_in,
                                                                const int32_t *__restrict__ idx_in, int64_t n,
                                                                int shift, int64_t ranges,
                                                                const int64_t *__restrict__ start,
                                                                uint32_t *__restrict__ key_out,
                                                                int32_t *__restrict__ idx_out)
{
    __shared__ uint32_t s_wc[kSortWaves][kRadix];   // per-wave digit counts, then offsets
    __shared__ int64_t s_base[kRadix];              // next slot of each digit for this range
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t r = blockIdx.x;
    for (int d = threadIdx.x; d < kRadix; d += blockDim.x) s_base[d] = start[(int64_t)d * ranges + r];
    const int64_t b = r * kRangeItems, e = min<int64_t>(n, b + kRangeItems);
    const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    for (int64_t c0 = b; c0 < e; c0 += kSortThreads) {
        for (int i = threadIdx.x; i < kSortWaves * kRadix; i += blockDim.x) (&s_wc[0][0])[i] = 0u;
        __syncthreads();
        const int64_t i = c0 + threadIdx.x;
        const bool valid = i < e;
        const uint32_t k = valid ? key_in[i] : 0u;
        const int32_t v = valid ? idx_in[i] : 0;
        const uint32_t dg = (k >> shift) & (kRadix - 1);
        // lanes of this wave holding the same digit: one ballot per bit
        uint64_t same = dev::ballot(valid);
#pragma unroll
        for (int bit = 0; bit < 8; bit++) {
            const bool one = (dg >> bit) & 1u;
            const uint64_t m = dev::ballot(one);
            same &= one ? m : ~m;
        }
        const int rank = __popcll(same & below);
        if (valid && rank == 0) s_wc[wave][dg] = (uint32_t)__popcll(same);
        __syncthreads();
        // per digit: exclusive prefix over the waves (offsets inside the chunk)
        for (int d = threadIdx.x; d < kRadix; d += blockDim.x) {
            uint32_t run = 0;
            for (int w = 0; w < kSortWaves; w++) {
                const uint32_t c = s_wc[w][d];
                s_wc[w][d] = run;
                run += c;
            }
            s_wc[0][d] |= run << 16;   // chunk total of digit d in the high half (at most 1,024)
        }
        __syncthreads();
        if (valid) {
            const uint32_t off = wave == 0 ? (s_wc[0][dg] & 0xffffu) : s_wc[wave][dg];
            const int64_t dst = s_base[dg] + off + rank;
            key_out[dst] = k;
            idx_out[dst] = v;
        }
        __syncthreads();
        for (int d = threadIdx.x; d < kRadix; d += blockDim.x) s_base[d] += s_wc[0][d] >> 16;
        __syncthreads();
    }
}

size_t sort_pairs_bytes(int64_t n)
{
    const int64_t ranges = std::max<int64_t>(1, (n + kRangeItems - 1) / kRangeItems);
    return (size_t)n * (sizeof(uint32_t) + sizeof(int32_t)) + (size_t)kRadix * ranges * sizeof(uint32_t) +
           ((size_t)kRadix * ranges + 1) * sizeof(int64_t) + 1024;
}

void sort_pairs_u32(uint32_t *keys, int32_t *vals, int64_t n, int bits, void *tmp, size_t tmp_bytes, hipStream_t st)
{
    if (n == 0 || bits <= 0) return;
    require(bits <= 32, "sort_pairs_u32: at most 32 key bits");
    require(tmp_bytes >= sort_pairs_bytes(n), "sort_pairs_u32: workspace too small");
    const int64_t ranges = std::max<int64_t>(1, (n + kRangeItems - 1) / kRangeItems);
    uint8_t *t = static_cast<uint8_t *>(tmp);
    uint32_t *k2 = reinterpret_cast<uint32_t *>(t);
    int32_t *v2 = reinterpret_cast<int32_t *>(k2 + n);
    uint32_t *hist = reinterpret_cast<uint32_t *>(v2 + n);
    int64_t *start = reinterpret_cast<int64_t *>(
        (reinterpret_cast<uintptr_t>(hist + (size_t)kRadix * ranges) + 7) & ~(uintptr_t)7);
    uint32_t *kbuf[2] = {keys, k2};
    int32_t *vbuf[2] = {vals, v2};
    const int passes = (bits + 7) / 8;
    int cur = 0;
    for (int p = 0; p < passes; p++) {
        hipLaunchKernelGGL(k_digit_hist, dim3((unsigned)ranges), dim3(kSortThreads), 0, st, kbuf[cur], n, 8 * p,
                           ranges, hist);
        check_launch("sort_pairs_u32(hist)");
        scan_u32(hist, kRadix * ranges, start, st);
        hipLaunchKernelGGL(k_digit_scatter, dim3((unsigned)ranges), dim3(kSortThreads), 0, st, kbuf[cur], vbuf[cur], n,
                           8 * p, ranges, start, kbuf[cur ^ 1], vbuf[cur ^ 1]);
        check_launch("sort_pairs_u32(scatter)");
        cur ^= 1;
    }
    if (cur == 1) {
        // an odd number of passes leaves the result in the workspace
        GTS_HIP(hipMemcpyAsync(keys, k2, (size_t)n * sizeof(uint32_t), hipMemcpyDeviceToDevice, st));
        GTS_HIP(hipMemcpyAsync(vals, v2, (size_t)n * sizeof(int32_t), hipMemcpyDeviceToDevice, st));
    }
}

static int key_bits(int64_t n_keys)
{
    int b = 1;
    while (b < 31 && ((int64_t)1 << b) < n_keys) b++;
    return b;
}

size_t home_sort_bytes(int64_t nq, int64_t n_keys)
{
    (void)n_keys;
    const int64_t ranges = std::max<int64_t>(1, (nq + kRangeItems - 1) / kRangeItems);
    // ping-pong indices, the digit table and its scan
    return (size_t)nq * sizeof(int32_t) * 2 + (size_t)kRadix * ranges * sizeof(uint32_t) +
           ((size_t)kRadix * ranges + 1) * sizeof(int64_t) + 1024;
}

void home_sort(const int32_t *home, int stride, int64_t nq, int64_t n_keys, uint32_t *keys, uint32_t *keys_sorted,
               int32_t *perm, void *tmp, size_t tmp_bytes, hipStream_t st)
{
    if (nq == 0) return;
    require(n_keys > 0 && n_keys < ((int64_t)1 << 31) && stride >= 1, "home_sort: key range out of bounds");
    require(tmp_bytes >= home_sort_bytes(nq, n_keys), "home_sort: workspace too small");
    const int64_t ranges = std::max<int64_t>(1, (nq + kRangeItems - 1) / kRangeItems);
    uint8_t *t = static_cast<uint8_t *>(tmp);
    int32_t *idx_a = reinterpret_cast<int32_t *>(t);
    int32_t *idx_b = idx_a + nq;
    uint32_t *hist = reinterpret_cast<uint32_t *>(idx_b + nq);
    int64_t *start = reinterpret_cast<int64_t *>(
        (reinterpret_cast<uintptr_t>(hist + (size_t)kRadix * ranges) + 7) & ~(uintptr_t)7);
    hipLaunchKernelGGL(k_home_keys, dim3((unsigned)((nq + 255) / 256)), dim3(256), 0, st, home, stride, nq, keys,
                       idx_a);
    check_launch(__func__);
    const int passes = (key_bits(n_keys) + 7) / 8;
    uint32_t *kbuf[2] = {keys, keys_sorted};
    int32_t *vbuf[2] = {idx_a, idx_b};
    int cur = 0;
    for (int p = 0; p < passes; p++) {
        // the last pass writes the permutation itself
        int32_t *vout = p == passes - 1 ? perm : vbuf[cur ^ 1];
        hipLaunchKernelGGL(k_digit_hist, dim3((unsigned)ranges), dim3(kSortThreads), 0, st, kbuf[cur], nq, 8 * p,
                           ranges, hist);
        check_launch("home_sort(hist)");
        scan_u32(hist, kRadix * ranges, start, st);
        hipLaunchKernelGGL(k_digit_scatter, dim3((unsigned)ranges), dim3(kSortThreads), 0, st, kbuf[cur], vbuf[cur],
                           nq, 8 * p, ranges, start, kbuf[cur ^ 1], vout);
        check_launch("home_sort(scatter)");
        cur ^= 1;
    }
}

}  // namespace k
}  // namespace gts
