// Device helpers shared by the kernels of libgts.so (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace gts {
namespace dev {

// ---------------------------------------------------------------------------
// bfloat16 (round to nearest even; inputs are finite)
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint16_t f32_to_bf16(float f)
{
    uint32_t u = __float_as_uint(f);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float bf16_to_f32(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// ---------------------------------------------------------------------------
// Wave primitives (wave64)
// ---------------------------------------------------------------------------
__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & 63u); }

__device__ __forceinline__ uint64_t ballot(bool p) { return (uint64_t)__ballot(p); }

// number of set bits of m below this lane
__device__ __forceinline__ int lanes_below(uint64_t m)
{
    return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// exclusive prefix sum over the wave; *total receives the wave sum
__device__ __forceinline__ int wave_excl_scan(int v, int *total)
{
    int lane = lane_id();
    int x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        int y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    *total = __shfl(x, 63, 64);
    return x - v;
}

// The distance an L2 computation reports: the Euclidean distance itself, or
// for the angular metric (both vectors of unit length) the angle between
// them, 2 asin(d / 2), which is monotone in d.
__device__ __forceinline__ float out_dist(float d, bool angular)
{
    return angular ? 2.f * asinf(fminf(0.5f * d, 1.f)) : d;
}

// One term of a direct-difference vector distance and the distance from the
// summed terms: (a - b)^2 and the square root for L2, |a - b| and the sum
// itself for L1 (Manhattan).
template <bool L1> __device__ __forceinline__ float dterm(float acc, float a, float b)
{
    const float d = a - b;
    return L1 ? acc + fabsf(d) : fmaf(d, d, acc);
}
template <bool L1> __device__ __forceinline__ float dfinish(float acc) { return L1 ? acc : sqrtf(acc); }
__device__ __forceinline__ float dterm_rt(bool l1, float acc, float a, float b)
{
    return l1 ? dterm<true>(acc, a, b) : dterm<false>(acc, a, b);
}
__device__ __forceinline__ float dfinish_rt(bool l1, float acc) { return l1 ? acc : sqrtf(acc); }

__device__ __forceinline__ float wave_min(float v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fminf(v, __shfl_xor(v, o, 64));
    return v;
}

// ---------------------------------------------------------------------------
// Levenshtein distance by bit-parallel vertical deltas (Myers 1999; the
// global-distance form where row 0 holds D[0][j] = j).  The pattern has up to
// 64*W characters.  Bytes are first mapped to alphabet codes by lut (the
// index's alphabet; bytes outside it share the last, all-zero row); peq[c*4+w]
// holds bit i of word w set iff pattern[64w+i] has code c.  Returns the exact
// distance when it is <= cutoff, otherwise some value > cutoff.
//
// Early exit: with m = plen and n = tlen, every alignment path crosses column
// j at some row i and still needs at least |(m - i) - (n - j)| operations;
// vertically adjacent cells differ by at most one, so the final distance is
// at least D[i*][j] on the row i* = j + m - n that ends on the last cell's
// diagonal.  That value is read off the vertical deltas every kChunk columns
// (the text characters of a chunk are loaded together, so a text in global
// memory costs one load latency per chunk, not per character).  The
// recurrences are host-callable too, so that they can be checked against the
// dynamic programme without a GPU.
// ---------------------------------------------------------------------------
template <int W, class PeqPtr>
__host__ __device__ __forceinline__ void myers_column(PeqPtr peq, int c, uint64_t (&VP)[W], uint64_t (&VN)[W], int topw,
                                             uint64_t topbit, int &score)
{
    uint64_t Xv[W], HP[W], HN[W];
    uint64_t carry = 0;
#pragma unroll
    for (int w = 0; w < W; w++) {
        const uint64_t Eq = peq[c * 4 + w];
        Xv[w] = Eq | VN[w];
        const uint64_t a = Eq & VP[w];
        const uint64_t s = a + VP[w];
        const uint64_t c1 = s < a ? 1ull : 0ull;
        const uint64_t s2 = s + carry;
        const uint64_t c2 = s2 < s ? 1ull : 0ull;
        carry = c1 | c2;
        const uint64_t Xh = (s2 ^ VP[w]) | Eq;
        HP[w] = VN[w] | ~(Xh | VP[w]);
        HN[w] = VP[w] & Xh;
    }
    uint64_t hp_top = 0, hn_top = 0;
#pragma unroll
    for (int w = 0; w < W; w++)
        if (w == topw) { hp_top = HP[w]; hn_top = HN[w]; }
    score += (hp_top & topbit) ? 1 : 0;
    score -= (hn_top & topbit) ? 1 : 0;
    // shift the horizontal deltas down one row; row 0 has delta +1
#pragma unroll
    for (int w = W - 1; w >= 0; w--) {
        const uint64_t inp = (w == 0) ? 1ull : (HP[w - 1] >> 63);
        const uint64_t inn = (w == 0) ? 0ull : (HN[w - 1] >> 63);
        HP[w] = (HP[w] << 1) | inp;
        HN[w] = (HN[w] << 1) | inn;
    }
#pragma unroll
    for (int w = 0; w < W; w++) {
        VP[w] = HN[w] | ~(Xv[w] | HP[w]);
        VN[w] = HP[w] & Xv[w];
    }
}

// D[i][j] of the current column j: D[0][j] = j plus the vertical deltas of
// rows 1..i (bit r of VP/VN is the delta from row r to row r+1).
template <int W>
__host__ __device__ __forceinline__ int myers_row_value(const uint64_t (&VP)[W], const uint64_t (&VN)[W], int j, int i)
{
    int v = j;
#pragma unroll
    for (int w = 0; w < W; w++) {
        const int bits = i - 64 * w;
        const uint64_t m = bits >= 64 ? ~0ull : (bits > 0 ? ((1ull << bits) - 1ull) : 0ull);
        v += __builtin_popcountll(VP[w] & m) - __builtin_popcountll(VN[w] & m);
    }
    return v;
}

template <int W, class PeqPtr, class LutPtr>
__host__ __device__ __forceinline__ int myers_distance(PeqPtr peq, int plen, const uint8_t *text, int tlen,
                                              int cutoff, LutPtr lut)
{
    if (plen == 0) return tlen;
    if (plen - tlen > cutoff || tlen - plen > cutoff) return cutoff + 1;
    uint64_t VP[W], VN[W];
#pragma unroll
    for (int w = 0; w < W; w++) {
        const int bits = plen - 64 * w;
        VP[w] = bits >= 64 ? ~0ull : (bits > 0 ? ((1ull << bits) - 1ull) : 0ull);
        VN[w] = 0ull;
    }
    const int topw = (plen - 1) >> 6;
    const uint64_t topbit = 1ull << ((plen - 1) & 63);
    int score = plen;
    constexpr int kChunk = 8;
    int j = 0;
    for (; j + kChunk <= tlen; j += kChunk) {
        int cs[kChunk];
#pragma unroll
        for (int u = 0; u < kChunk; u++) cs[u] = lut[text[j + u]];
#pragma unroll
        for (int u = 0; u < kChunk; u++) myers_column<W>(peq, cs[u], VP, VN, topw, topbit, score);
        const int is = j + kChunk + plen - tlen;   // in (.., plen]
        if (is > 0 && myers_row_value<W>(VP, VN, j + kChunk, is) > cutoff) return cutoff + 1;
    }
    for (; j < tlen; j++) myers_column<W>(peq, lut[text[j]], VP, VN, topw, topbit, score);
    return score;
}

// Banded form for cutoffs k <= 63: one word of B bits whatever the pattern
// length (B = 32 for k <= 31, else 64).  An alignment of cost <= k only
// visits diagonals j - i in [lo, hi] with |j - i| + |j - i - (n - m)| <= k,
// at most k + 1 <= B of them, so a window of B consecutive rows that moves
// down one row per column (top row r_j = max(1, j - hi)) holds every cell
// such an alignment visits.  Cells outside
// the window enter as upper bounds (vertical delta +1 below it, horizontal
// delta +1 above it, no carry from above), so every computed value is at
// least the true one and equals it for a cell whose optimal alignment stays
// in the band: the result is exact when it is <= k and above k otherwise.
// The value of the window's top cell is carried from column to column; the
// early exit reads the cell on the last cell's diagonal as in
// myers_distance.  nw = words per code held by peq (bits past the pattern
// are zero).
template <class T, class PeqPtr, class LutPtr>
__host__ __device__ __forceinline__ int myers_banded_w(PeqPtr peq, int nw, int plen, const uint8_t *text, int tlen,
                                                       int cutoff, LutPtr lut)
{
    constexpr int B = 8 * (int)sizeof(T);   // window rows; requires cutoff <= B - 1
    if (plen == 0) return tlen;
    const int delta = tlen - plen;
    const int ad = delta < 0 ? -delta : delta;
    if (ad > cutoff) return cutoff + 1;
    const int hi = (delta > 0 ? delta : 0) + ((cutoff - ad) >> 1);   // top diagonal of the band
    const int tstar = hi - delta;   // window bit of the last cell's diagonal once the window moves
    T VP = (T)~(T)0, VN = 0;
    int top = 1;   // D[r_j][j]; before the first column D[1][0] = 1
    auto column = [&](int j, int c) {   // j: 1-based column
        // branch-free: the window moves (sft = 1) once j > hi + 1; both table
        // words are loaded from clamped indexes and zeroed past the table
        const int sft = j > hi + 1 ? 1 : 0;
        VP = (T)((VP >> sft) | ((T)sft << (B - 1)));
        VN >>= sft;
        const int s0 = min(max(0, j - hi - 1), 255);   // 0-based pattern index of the top row (texts <= 255)
        const int w0 = s0 >> 6, sh = s0 & 63;
        uint64_t a = peq[c * 4 + min(w0, nw - 1)];
        uint64_t b = peq[c * 4 + min(w0 + 1, nw - 1)];
        a = w0 < nw ? a : 0ull;
        b = w0 + 1 < nw ? b : 0ull;
        const T Eq = (T)((a >> sh) | ((b << 1) << (63 - sh)));   // bits s0 .. s0+B-1
        const T Xv = Eq | VN;
        const T Xh = (T)((T)((Eq & VP) + VP) ^ VP) | Eq;
        T HP = (T)(VN | (T)~(Xh | VP));
        T HN = VP & Xh;
        HP = (T)((T)(HP << 1) | (T)1);
        HN = (T)(HN << 1);
        VP = (T)(HN | (T)~(Xv | HP));
        VN = HP & Xv;
        const int vd0 = (int)(VP & (T)1) - (int)(VN & (T)1);
        top = (sft ? top + 1 : j) + vd0;
    };
    // D[r_j + t][j] - D[r_j][j] for t in 1..B-1
    auto below = [&](int t) {
        const T m = (T)((T)((T)2 << t) - (T)2);
        return __builtin_popcountll((uint64_t)(VP & m)) - __builtin_popcountll((uint64_t)(VN & m));
    };
    constexpr int kChunk = 8;
    int j = 0;
    for (; j + kChunk <= tlen; j += kChunk) {
        int cs[kChunk];
#pragma unroll
        for (int u = 0; u < kChunk; u++) cs[u] = lut[text[j + u]];
#pragma unroll
        for (int u = 0; u < kChunk; u++) column(j + u + 1, cs[u]);
        const int jj = j + kChunk;
        const int t = jj > hi + 1 ? tstar : jj - delta - 1;   // the last cell's diagonal in the window
        if (t >= 0 && top + (t > 0 ? below(t) : 0) > cutoff) return cutoff + 1;
    }
    for (; j < tlen; j++) column(j + 1, lut[text[j]]);
    const int rn = tlen > hi + 1 ? tlen - hi : 1;
    const int tm = plen - rn;
    const int d = top + (tm > 0 ? below(tm) : 0);
    return d <= cutoff ? d : cutoff + 1;
}

template <class PeqPtr, class LutPtr>
__host__ __device__ __forceinline__ int myers_banded(PeqPtr peq, int nw, int plen, const uint8_t *text, int tlen,
                                                     int cutoff, LutPtr lut)
{
    if (cutoff <= 31) return myers_banded_w<uint32_t>(peq, nw, plen, text, tlen, cutoff, lut);
    return myers_banded_w<uint64_t>(peq, nw, plen, text, tlen, cutoff, lut);
}

template <class PeqPtr, class LutPtr>
__device__ __forceinline__ int myers_any(PeqPtr peq, int plen, const uint8_t *text, int tlen, int cutoff, LutPtr lut)
{
    if (cutoff <= 63) return myers_banded(peq, 4, plen, text, tlen, cutoff, lut);
    if (plen <= 64) return myers_distance<1>(peq, plen, text, tlen, cutoff, lut);
    if (plen <= 128) return myers_distance<2>(peq, plen, text, tlen, cutoff, lut);
    if (plen <= 192) return myers_distance<3>(peq, plen, text, tlen, cutoff, lut);
    return myers_distance<4>(peq, plen, text, tlen, cutoff, lut);
}

// Set the match bits of one pattern in a table of `rows` codes (zeroed by the
// caller); bytes outside the alphabet (code rows-1) set nothing, so they match
// no text byte.  Threads stride over the pattern; atomic OR on the table.
template <class Tab>
__device__ __forceinline__ void peq_fill(Tab tab, const uint8_t *pat, int plen, const uint8_t *lut, int rows)
{
    for (int b = threadIdx.x; b < plen; b += blockDim.x) {
        const int c = lut[pat[b]];
        if (c < rows - 1)
            atomicOr(reinterpret_cast<unsigned long long *>(&tab[c * 4 + (b >> 6)]),
                     (unsigned long long)(1ull << (b & 63)));
    }
}

// ---------------------------------------------------------------------------
// Bitonic sort of n (a power of two) 64-bit keys, ascending, by the whole
// workgroup.  Works on LDS or global memory; begins and ends with a barrier.
// ---------------------------------------------------------------------------
template <class T>
__device__ void bitonic_sort(T *a, int n)
{
    for (int size = 2; size <= n; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            __syncthreads();
            for (int i = threadIdx.x; i < (n >> 1); i += blockDim.x) {
                int lo = 2 * i - (i & (stride - 1));
                int hi = lo + stride;
                bool up = (lo & size) == 0;
                T x = a[lo], y = a[hi];
                if ((x > y) == up) {
                    a[lo] = y;
                    a[hi] = x;
                }
            }
        }
    }
    __syncthreads();
}

__device__ __forceinline__ int next_pow2(int v)
{
    int p = 1;
    while (p < v) p <<= 1;
    return p;
}

// Bitonic sort of n (a power of two) keys in LDS by one wave (lanes in
// lockstep: a wave barrier orders the passes).
__device__ inline void wave_bitonic_sort(uint64_t *a, int n)
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

// Sort keys[0, nk) by the workgroup (padded with ~0 to a power of two within
// cap), then write the first min(k, nk) (k > 0) or all nk to out and the
// count to *out_count_q.
__device__ inline void sort_and_emit(uint64_t *keys, int nk, int64_t cap, int k, uint64_t *out, uint32_t *out_count_q)
{
    const int P = next_pow2(nk > 1 ? nk : 1);
    for (int i = nk + threadIdx.x; i < P && i < cap; i += blockDim.x) keys[i] = ~0ull;
    bitonic_sort(keys, P);
    const int nout = (k > 0 && k < nk) ? k : nk;
    for (int j = threadIdx.x; j < nout; j += blockDim.x) out[j] = keys[j];
    if (threadIdx.x == 0) *out_count_q = (uint32_t)nout;
}

}  // namespace dev
}  // namespace gts
