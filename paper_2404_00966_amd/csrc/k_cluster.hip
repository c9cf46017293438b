// Build-time clustering that orders the objects before they are cut into
// leaves.
//
// The centres come from farthest-first traversal (the pivot selection rule of
// Algorithm 2, Sec. 4.3, run to many more centres): centre j + 1 is
// the object farthest from centres 0..j.  One launch per centre; each launch
// reads the previous argmax from device memory and leaves its own argmax
// there, so the K launches run back to back without host round trips.
//
// Key of an object: (bits of its distance to the nearest centre so far) << 32
// | (0xffffffff - index); the largest key is the farthest object, ties going
// to the smallest index.  Distances are >= 0, so their float bits order as
// unsigned integers.
#include "dev_common.h"
#include "kernels.h"

namespace gts {
namespace k {

namespace {

__device__ __forceinline__ uint64_t far_key(float d, int64_t i)
{
    return ((uint64_t)__float_as_uint(d) << 32) | (uint64_t)(0xffffffffu - (uint32_t)i);
}

__device__ __forceinline__ int64_t key_index(uint64_t k) { return (int64_t)(0xffffffffu - (uint32_t)k); }

// block-wide max of a 64-bit key, then one atomic per block
__device__ __forceinline__ void block_max_atomic(uint64_t v, uint64_t *dst)
{
    __shared__ uint64_t s_w[16];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const uint64_t u = __shfl_xor(v, o, 64);
        v = u > v ? u : v;
    }
    const int wave = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) s_w[wave] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t m = 0;
        for (int w = 0; w < (int)(blockDim.x >> 6); w++) m = s_w[w] > m ? s_w[w] : m;
        atomicMax(reinterpret_cast<unsigned long long *>(dst), (unsigned long long)m);
    }
}

}  // namespace

// Step j (L2): squared distance of every object to centre c_j = the argmax
// left in keys[j]; nearest-centre bookkeeping; argmax into keys[j + 1].
__global__ __launch_bounds__(256) void k_fft_step_l2(const float *__restrict__ X, int64_t n, int dp, int j,
                                                     uint64_t *__restrict__ keys, int32_t *__restrict__ centers,
                                                     float *__restrict__ mind, int32_t *__restrict__ near, int l1)
{
    const int64_t c = key_index(keys[j]);
    if (blockIdx.x == 0 && threadIdx.x == 0) centers[j] = (int32_t)c;
    const int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    uint64_t key = 0;
    if (o < n) {
        const float4 *x = reinterpret_cast<const float4 *>(X + (size_t)o * dp);
        const float4 *y = reinterpret_cast<const float4 *>(X + (size_t)c * dp);
        float a0 = 0.f, a1 = 0.f, a2 = 0.f, a3 = 0.f;
        if (l1) {
            for (int i = 0; i < dp / 4; i++) {
                const float4 u = x[i], v = y[i];
                a0 = dev::dterm<true>(a0, u.x, v.x);
                a1 = dev::dterm<true>(a1, u.y, v.y);
                a2 = dev::dterm<true>(a2, u.z, v.z);
                a3 = dev::dterm<true>(a3, u.w, v.w);
            }
        } else {
            for (int i = 0; i < dp / 4; i++) {
                const float4 u = x[i], v = y[i];
                a0 = dev::dterm<false>(a0, u.x, v.x);
                a1 = dev::dterm<false>(a1, u.y, v.y);
                a2 = dev::dterm<false>(a2, u.z, v.z);
                a3 = dev::dterm<false>(a3, u.w, v.w);
            }
        }
        const float d = (a0 + a1) + (a2 + a3);   // squared for L2 (the order is the same)
        float m = mind[o];
        if (j == 0 || d < m) {
            m = d;
            mind[o] = d;
            near[o] = j;
        }
        key = far_key(m, o);
    }
    block_max_atomic(key, keys + j + 1);
}

// Step j (edit distance): the centre string is the Myers pattern (its match
// table in LDS); an object's distance only matters when it is below its
// current nearest-centre distance, which is the early-exit cutoff.
__global__ __launch_bounds__(256) void k_fft_step_edit(const uint8_t *__restrict__ chars,
                                                       const int64_t *__restrict__ off, int64_t n,
                                                       const uint8_t *__restrict__ lut_g, int arows, int j,
                                                       uint64_t *__restrict__ keys, int32_t *__restrict__ centers,
                                                       float *__restrict__ mind, int32_t *__restrict__ near)
{
    __shared__ uint64_t s_peq[257 * 4];
    __shared__ uint8_t s_lut[256];
    const int64_t c = key_index(keys[j]);
    if (blockIdx.x == 0 && threadIdx.x == 0) centers[j] = (int32_t)c;
    for (int i = threadIdx.x; i < arows * 4; i += blockDim.x) s_peq[i] = 0ull;
    for (int i = threadIdx.x; i < 256; i += blockDim.x) s_lut[i] = lut_g[i];
    __syncthreads();
    const int64_t ca = off[c];
    const int plen = (int)(off[c + 1] - ca);
    dev::peq_fill(s_peq, chars + ca, plen, s_lut, arows);
    __syncthreads();
    const int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    uint64_t key = 0;
    if (o < n) {
        float m = mind[o];
        const int cutoff = j == 0 ? (1 << 30) : (int)m - 1;
        if (cutoff >= 0) {
            const int64_t a = off[o];
            const int d = dev::myers_any(s_peq, plen, chars + a, (int)(off[o + 1] - a), cutoff, s_lut);
            if (d <= cutoff) {
                m = (float)d;
                mind[o] = m;
                near[o] = j;
            }
        }
        key = far_key(m, o);
    }
    block_max_atomic(key, keys + j + 1);
}

void fft_centers_l2(const float *X, int64_t n, int dp, int K, uint64_t *keys, int32_t *centers, float *mind,
                    int32_t *near, hipStream_t st, bool l1)
{
    const unsigned grid = (unsigned)((n + 255) / 256);
    for (int j = 0; j < K; j++)
        hipLaunchKernelGGL(k_fft_step_l2, dim3(grid), dim3(256), 0, st, X, n, dp, j, keys, centers, mind, near,
                           l1 ? 1 : 0);
    check_launch(__func__);
}

void fft_centers_edit(const uint8_t *chars, const int64_t *off, int64_t n, const uint8_t *lut, int arows, int K,
                      uint64_t *keys, int32_t *centers, float *mind, int32_t *near, hipStream_t st)
{
    const unsigned grid = (unsigned)((n + 255) / 256);
    for (int j = 0; j < K; j++)
        hipLaunchKernelGGL(k_fft_step_edit, dim3(grid), dim3(256), 0, st, chars, off, n, lut, arows, j, keys,
                           centers, mind, near);
    check_launch(__func__);
}

}  // namespace k
}  // namespace gts
