// Preparation kernels: bf16 MFMA fragments of object / query rows with their
// norms and rounding errors, distances to pivots (both metrics), and the
// match-bit tables of query strings.
#include "dev_common.h"
#include "kernels.h"

namespace gts {
namespace k {

// One thread per row.  Writes the row rounded to bf16 in the MFMA fragment
// layout [row/16][kstep][lane][8] where lane = row%16 + 16*g holds columns
// 32*kstep + 8*g .. +7 (zero beyond dim), plus ||x16||^2 and ||x16 - x||.
// Rows >= rows_valid are padding: zero fragments, norm2 = pad_norm2, err = 0.
__global__ void k_rows_bf16(const float *__restrict__ X, int64_t rows_valid, int64_t rows_pad, int dim,
                            int stride, int ksteps, uint16_t *__restrict__ frag, float *__restrict__ norm2,
                            float *__restrict__ err, float pad_norm2)
{
    int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= rows_pad) return;
    const bool valid = r < rows_valid;
    const float *x = X + (size_t)r * stride;
    float n2 = 0.f, e2 = 0.f;
    const int64_t g = r >> 4;
    const int rr = (int)(r & 15);
    for (int s = 0; s < ksteps; s++) {
        for (int q4 = 0; q4 < 4; q4++) {
            uint16_t h[8];
#pragma unroll
            for (int e = 0; e < 8; e++) {
                int c = 32 * s + 8 * q4 + e;
                float v = (valid && c < dim) ? x[c] : 0.f;
                h[e] = dev::f32_to_bf16(v);
                float b = dev::bf16_to_f32(h[e]);
                n2 = fmaf(b, b, n2);
                float d = b - v;
                e2 = fmaf(d, d, e2);
            }
            uint4 packed;
            packed.x = (uint32_t)h[0] | ((uint32_t)h[1] << 16);
            packed.y = (uint32_t)h[2] | ((uint32_t)h[3] << 16);
            packed.z = (uint32_t)h[4] | ((uint32_t)h[5] << 16);
            packed.w = (uint32_t)h[6] | ((uint32_t)h[7] << 16);
            size_t lane = (size_t)(rr + 16 * q4);
            *reinterpret_cast<uint4 *>(frag + (((size_t)g * ksteps + s) * 64 + lane) * 8) = packed;
        }
    }
    norm2[r] = valid ? n2 : pad_norm2;
    err[r] = valid ? sqrtf(e2) : 0.f;
}

void rows_bf16(const float *X, int64_t rows_valid, int64_t rows_pad, int dim, int stride, int ksteps,
               uint16_t *frag, float *norm2, float *err, float pad_norm2, hipStream_t st)
{
    if (rows_pad == 0) return;
    int blocks = (int)((rows_pad + 255) / 256);
    hipLaunchKernelGGL(k_rows_bf16, dim3(blocks), dim3(256), 0, st, X, rows_valid, rows_pad, dim, stride,
                       ksteps, frag, norm2, err, pad_norm2);
    check_launch(__func__);
}

// out[i * s_piv + r * s_row] = || X[r] - P[i] ||  (float32, direct difference,
// rows of both padded to `stride` floats).  16 lanes per (row, pivot) pair,
// each summing a strided slice of the coordinates (coalesced 64-byte runs),
// then a 16-lane reduction.  Columns i in [m, mpad) get 0.
__global__ __launch_bounds__(256) void k_dist_l2_pivots(const float *__restrict__ X, int64_t rows,
                                                        const float *__restrict__ P, int m, int mpad, int stride,
                                                        float *__restrict__ out, int64_t s_piv, int64_t s_row,
                                                        int l1)
{
    const int64_t g = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 4;
    const int sl = threadIdx.x & 15;
    const int64_t r = g / mpad;
    const int i = (int)(g % mpad);
    const bool ok = r < rows;
    float acc = 0.f;
    if (ok && i < m) {
        const float *x = X + (size_t)r * stride;
        const float *p = P + (size_t)i * stride;
        if (l1)
            for (int c = sl; c < stride; c += 16) acc = dev::dterm<true>(acc, x[c], p[c]);
        else
            for (int c = sl; c < stride; c += 16) acc = dev::dterm<false>(acc, x[c], p[c]);
    }
#pragma unroll
    for (int o = 8; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 16);
    if (ok && sl == 0) out[(size_t)i * s_piv + (size_t)r * s_row] = i < m ? dev::dfinish_rt(l1 != 0, acc) : 0.f;
}

void dist_l2_pivots(const float *X, int64_t rows, const float *P, int m, int mpad, int stride, float *out,
                    int64_t s_piv, int64_t s_row, hipStream_t st, bool l1)
{
    if (rows == 0) return;
    const int64_t threads = rows * mpad * 16;
    hipLaunchKernelGGL(k_dist_l2_pivots, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, st, X, rows, P, m,
                       mpad, stride, out, s_piv, s_row, l1 ? 1 : 0);
    check_launch(__func__);
}

// Edit distance of every string to pivot blockIdx.y: the pivot is the Myers
// pattern (its match table in LDS), each thread scans one string as the text.
// out[i * s_piv + r * s_row] = distance.
__global__ void k_dist_edit_pivots(const uint8_t *__restrict__ chars, const int64_t *__restrict__ off,
                                   int64_t rows, const uint8_t *__restrict__ pchars, const int32_t *__restrict__ poff,
                                   int m, float *__restrict__ out, int64_t s_piv, int64_t s_row,
                                   const uint8_t *__restrict__ lut_g, int arows)
{
    __shared__ uint64_t peq[257 * 4];
    __shared__ uint8_t lut[256];
    const int i = blockIdx.y;
    for (int t = threadIdx.x; t < arows * 4; t += blockDim.x) peq[t] = 0ull;
    for (int t = threadIdx.x; t < 256; t += blockDim.x) lut[t] = lut_g[t];
    __syncthreads();
    int plen = 0;
    if (i < m) {
        const int a = poff[i];
        plen = poff[i + 1] - a;
        dev::peq_fill(peq, pchars + a, plen, lut, arows);
    }
    __syncthreads();
    int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= rows) return;
    int d = 0;
    if (i < m) {
        const int64_t a = off[r];
        const int tlen = (int)(off[r + 1] - a);
        d = dev::myers_any(peq, plen, chars + a, tlen, 1 << 30, lut);
    }
    out[(size_t)i * s_piv + (size_t)r * s_row] = (float)d;
}

void dist_edit_pivots_f32(const uint8_t *chars, const int64_t *off, int64_t rows, const uint8_t *pchars,
                          const int32_t *poff, int m, int mpad, float *out, int64_t s_piv, int64_t s_row,
                          const uint8_t *lut, int arows, hipStream_t st)
{
    if (rows == 0) return;
    dim3 grid((unsigned)((rows + 255) / 256), (unsigned)mpad);
    hipLaunchKernelGGL(k_dist_edit_pivots, grid, dim3(256), 0, st, chars, off, rows, pchars, poff, m, out, s_piv,
                       s_row, lut, arows);
    check_launch(__func__);
}

// Match-bit table of each query string over the index alphabet:
// peq[q][c][w] bit b set iff query[64w + b] has code c.  One workgroup per
// query.
__global__ void k_build_peq(const uint8_t *__restrict__ chars, const int64_t *__restrict__ off, int64_t nq,
                            const uint8_t *__restrict__ lut, int arows, uint64_t *__restrict__ peq)
{
    int64_t q = blockIdx.x;
    if (q >= nq) return;
    uint64_t *t = peq + (size_t)q * arows * 4;
    for (int c = threadIdx.x; c < arows * 4; c += blockDim.x) t[c] = 0ull;
    __syncthreads();
    const int64_t a = off[q];
    dev::peq_fill(t, chars + a, (int)(off[q + 1] - a), lut, arows);
}

void build_peq(const uint8_t *chars, const int64_t *off, int64_t nq, const uint8_t *lut, int arows, uint64_t *peq,
               hipStream_t st)
{
    if (nq == 0) return;
    hipLaunchKernelGGL(k_build_peq, dim3((unsigned)nq), dim3(256), 0, st, chars, off, nq, lut, arows, peq);
    check_launch(__func__);
}

// Per-query thresholds for node and object filtering:
//   L2:   thr = T + 2*delta*(max_i QP[q][i] + pt_max), T = base * (1 + 2*delta)
//         cut = base (range) or T (kNN): the float32-distance emission cutoff
//   EDIT: thr = T = cut = floor(base)
// where base is the range radius or the kNN bound and delta bounds the
// relative float32 error of a direct-difference distance in `dim` dimensions.
__global__ void k_thresholds(const float *__restrict__ base, const float *__restrict__ QP, const int32_t *__restrict__ kq,
                             int64_t nq, int mpad, int is_edit, float delta, float pt_max, float *__restrict__ T,
                             float *__restrict__ thr, float *__restrict__ cut)
{
    int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= nq) return;
    float b = base[q];
    if (is_edit) {
        float t = floorf(fminf(b, 1e6f));
        T[q] = t;
        thr[q] = t;
        cut[q] = t;
        return;
    }
    float qmax = 0.f;
    for (int i = 0; i < mpad; i++) qmax = fmaxf(qmax, QP[(size_t)q * mpad + i]);
    float t = b * (1.f + 2.f * delta);
    T[q] = t;
    thr[q] = t + 2.f * delta * (qmax + pt_max);
    cut[q] = kq[q] > 0 ? t : b;
}

void thresholds(const float *base, const float *QP, const int32_t *kq, int64_t nq, int mpad, int is_edit, float delta,
                float pt_max, float *T, float *thr, float *cut, hipStream_t st)
{
    if (nq == 0) return;
    hipLaunchKernelGGL(k_thresholds, dim3((unsigned)((nq + 255) / 256)), dim3(256), 0, st, base, QP, kq, nq, mpad,
                       is_edit, delta, pt_max, T, thr, cut);
    check_launch(__func__);
}

// *bad |= 1 when any of the first dim values of the rows is not finite;
// such a value is replaced by zero, so that no later kernel reads it.
__global__ void k_check_finite(float *__restrict__ X, int64_t rows, int dim, int stride, uint32_t *__restrict__ bad)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= rows * dim) return;
    const int64_t r = i / dim;
    const int c = (int)(i - r * dim);
    float *x = X + (size_t)r * stride + c;
    if (!isfinite(*x)) {
        *x = 0.f;
        atomicOr(bad, 1u);
    }
}

void check_finite(float *X, int64_t rows, int dim, int stride, uint32_t *bad, hipStream_t st)
{
    const int64_t n = rows * dim;
    if (n == 0) return;
    hipLaunchKernelGGL(k_check_finite, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, X, rows, dim, stride, bad);
    check_launch(__func__);
}

// Per-query parameters of a graph-replayed search from device arrays: kq =
// k (>= 1: kNN), base = the range radius (the chord 2 sin(r / 2) for the
// angular metric) where k == 0; a negative k or a negative or NaN radius
// sets bit 1 of *status (that query is then run as a range query of radius 0).
__global__ void k_query_params(const float *__restrict__ radius, const int32_t *__restrict__ k, int64_t nq,
                               int angular, float *__restrict__ base, int32_t *__restrict__ kq,
                               uint32_t *__restrict__ status)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= nq) return;
    const int kk = k[q];
    bool bad = kk < 0;
    float b = 0.f;
    if (kk <= 0) {
        const float r = radius[q];
        if (!(r >= 0.f) || !isfinite(r)) bad = true;
        else b = angular ? (float)(2.0 * sin(fmin((double)r, 3.141592653589793) / 2.0)) : r;
    }
    kq[q] = kk > 0 ? kk : 0;
    base[q] = b;
    if (bad) atomicOr(status, 1u);
}

void query_params(const float *radius, const int32_t *k, int64_t nq, bool angular, float *base, int32_t *kq,
                  uint32_t *status, hipStream_t st)
{
    if (nq == 0) return;
    hipLaunchKernelGGL(k_query_params, dim3((unsigned)((nq + 255) / 256)), dim3(256), 0, st, radius, k, nq,
                       angular ? 1 : 0, base, kq, status);
    check_launch(__func__);
}

// The status word of a graph-replayed search, after its last kernel: bit 2
// for a bad query (a non-finite value, or a zero vector of the angular
// metric), bit 4 when the candidates exceeded their space, bit 8 when the
// answers exceeded the output capacity.
__global__ void k_plan_status(uint32_t *__restrict__ status, const uint32_t *__restrict__ bad_query,
                              const unsigned long long *__restrict__ cand_count, int64_t cand_cap,
                              const int64_t *__restrict__ total, int64_t answer_cap)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    uint32_t s = *status;
    if (bad_query && *bad_query) s |= 2u;
    if (cand_count && *cand_count > (unsigned long long)cand_cap) s |= 4u;
    if (total && *total > answer_cap) s |= 8u;
    *status = s;
}

void plan_status(uint32_t *status, const uint32_t *bad_query, const unsigned long long *cand_count, int64_t cand_cap,
                 const int64_t *total, int64_t answer_cap, hipStream_t st)
{
    hipLaunchKernelGGL(k_plan_status, dim3(1), dim3(64), 0, st, status, bad_query, cand_count, cand_cap, total,
                       answer_cap);
    check_launch(__func__);
}

// Unit rows for the angular metric: one wave per row, the squared norm
// summed in double over the lanes, every coordinate divided by the norm in
// double and rounded to float (within one rounding of the true unit vector).
__global__ __launch_bounds__(256) void k_normalize_rows(float *__restrict__ X, int64_t rows, int dim, int stride,
                                                        uint32_t *__restrict__ bad)
{
    const int64_t r = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int lane = threadIdx.x & 63;
    if (r >= rows) return;
    float *x = X + (size_t)r * stride;
    double acc = 0.0;
    for (int i = lane; i < dim; i += 64) acc += (double)x[i] * (double)x[i];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
    const double nrm = sqrt(acc);
    const bool ok = nrm > 0.0 && nrm < INFINITY;
    for (int i = lane; i < dim; i += 64) x[i] = ok ? (float)((double)x[i] / nrm) : 0.f;
    if (!ok && lane == 0) atomicOr(bad, 1u);
}

void normalize_rows(float *X, int64_t rows, int dim, int stride, uint32_t *bad, hipStream_t st)
{
    if (rows == 0) return;
    hipLaunchKernelGGL(k_normalize_rows, dim3((unsigned)((rows + 3) / 4)), dim3(256), 0, st, X, rows, dim, stride,
                       bad);
    check_launch(__func__);
}

__global__ void k_scatter_u32(uint32_t *__restrict__ dst, const uint32_t *__restrict__ at,
                              const uint32_t *__restrict__ val, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[at[i]] = val[i];
}

void scatter_u32(uint32_t *dst, const uint32_t *at, const uint32_t *val, int64_t n, hipStream_t st)
{
    if (n == 0) return;
    hipLaunchKernelGGL(k_scatter_u32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, dst, at, val, n);
    check_launch(__func__);
}

// Tombstone bitmap of one epoch: bit p of bits[] is set iff position p was
// deleted by an update of epoch e or earlier (del_ep[p] <= e; a live position
// holds 0xffffffff).  One lane per position, the wave's 64 decisions made
// into two words by one ballot; words past n hold zeros.
__global__ void k_tomb_bits(const uint32_t *__restrict__ del_ep, int64_t n, uint32_t e, uint32_t *__restrict__ bits,
                            int64_t words)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool dead = p < n && del_ep[p] <= e;
    const uint64_t m = dev::ballot(dead);
    const int lane = dev::lane_id();
    const int64_t w0 = (p - lane) >> 5;   // first of this wave's two words
    if (lane == 0 && w0 < words) bits[w0] = (uint32_t)m;
    if (lane == 32 && w0 + 1 < words) bits[w0 + 1] = (uint32_t)(m >> 32);
}

void tomb_bits(const uint32_t *del_ep, int64_t n, uint32_t e, uint32_t *bits, int64_t words, hipStream_t st)
{
    if (words == 0) return;
    const int64_t threads = (words * 32 + 255) / 256 * 256;
    hipLaunchKernelGGL(k_tomb_bits, dim3((unsigned)(threads / 256)), dim3(256), 0, st, del_ep, n, e, bits, words);
    check_launch(__func__);
}

// Work of each query tile: out[t] += sum over leaves of (queries of the
// tile that keep the leaf) x (objects of the leaf), from the (leaf, tile)
// masks [n_leaves][ntiles].  out must start at zero.
__global__ void k_tile_pairs(const uint64_t *__restrict__ mask, int64_t n_leaves, int ntiles,
                             const int32_t *__restrict__ leaf_cnt, unsigned long long *__restrict__ out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_leaves * ntiles) return;
    const int64_t leaf = i / ntiles;
    const int t = (int)(i - leaf * ntiles);
    const uint64_t m = mask[i];
    if (m) atomicAdd(&out[t], (unsigned long long)__popcll(m) * (unsigned long long)leaf_cnt[leaf]);
}

void tile_pairs(const uint64_t *mask, int64_t n_leaves, int ntiles, const int32_t *leaf_cnt, unsigned long long *out,
                hipStream_t st)
{
    const int64_t n = n_leaves * ntiles;
    if (n == 0) return;
    hipLaunchKernelGGL(k_tile_pairs, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, mask, n_leaves, ntiles,
                       leaf_cnt, out);
    check_launch(__func__);
}

// out[q] = a[q] + b[q] for q < n, -inf for n <= q < npad (padding rows of a
// query tile never pass a threshold).
__global__ void k_sum_pad(const float *__restrict__ a, const float *__restrict__ b, int64_t n, int64_t npad,
                          float *__restrict__ out)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= npad) return;
    out[q] = q < n ? a[q] + b[q] : -INFINITY;
}

void sum_pad(const float *a, const float *b, int64_t n, int64_t npad, float *out, hipStream_t st)
{
    if (npad == 0) return;
    hipLaunchKernelGGL(k_sum_pad, dim3((unsigned)((npad + 255) / 256)), dim3(256), 0, st, a, b, n, npad, out);
    check_launch(__func__);
}

// Fill an int32 / uint64 array (a small kernel, so no memset node is needed
// when the stream is captured).
__global__ void k_fill_u32(uint32_t *p, int64_t n, uint32_t v)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

void fill_u32(uint32_t *p, int64_t n, uint32_t v, hipStream_t st)
{
    if (n <= 0) return;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)blocks), dim3(256), 0, st, p, n, v);
    check_launch(__func__);
}

}  // namespace k
}  // namespace gts
