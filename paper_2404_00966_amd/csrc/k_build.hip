// Device steps of the L2 index construction (Sec. 4.3): the object table,
// the pivot table and every per-node summary are formed in HBM from the
// objects in input order and the leaf order, without host round trips of
// n-sized arrays.
//
//   k_gather_rows    : rows into a new order (float4 copies)
//   k_gather_pt      : pivot-table columns into leaf order
//   k_nearest_centre : every object's nearest centre (exact float32)
//   k_centre_dist    : squared distance of each object to its cell's centre
//   k_cell_keys      : per position, the chain rank of the object's cell
//   k_leaf_boxes     : per leaf, per pivot row, min and max of the table
//   k_node_boxes     : a node's box from its children's (one level)
//   k_box_soa        : node boxes also as pivot-major lo / hi rows
//   k_slab_summary   : per 256-row slab, the largest bf16 rounding error and
//                      norm, and the leaves it overlaps
//   k_leaf_centroid  : per leaf, the mean of its objects (double)
//   k_leaf_pivot     : per leaf, the object nearest the mean and the largest
//                      distance from it to the leaf's objects (double)
//   k_max_f32        : largest value of a non-negative float array
#include "dev_common.h"
#include "gts_internal.h"
#include "kernels.h"

namespace gts {
namespace k {

__global__ void k_gather_rows(const float4 *__restrict__ src, const int32_t *__restrict__ perm, int64_t n, int q4,
                              float4 *__restrict__ dst)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n * q4) return;
    const int64_t p = i / q4;
    const int c = (int)(i - p * q4);
    dst[i] = src[(int64_t)perm[p] * q4 + c];
}

void gather_rows(const float *src, int dp, const int32_t *perm, int64_t n, float *dst, hipStream_t st)
{
    if (n == 0) return;
    require(dp % 4 == 0, "gather_rows: row stride not a multiple of 4 floats");
    const int64_t threads = n * (dp / 4);
    hipLaunchKernelGGL(k_gather_rows, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, st,
                       reinterpret_cast<const float4 *>(src), perm, n, dp / 4, reinterpret_cast<float4 *>(dst));
    check_launch(__func__);
}

// dst[i][p] = src[i][perm[p]] for i < m, 0 for m <= i < mpad (rows of n).
__global__ void k_gather_pt(const float *__restrict__ src, const int32_t *__restrict__ perm, int64_t n, int m,
                            int mpad, float *__restrict__ dst)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const int64_t o = perm[p];
    for (int i = 0; i < mpad; i++) dst[(size_t)i * n + p] = i < m ? src[(size_t)i * n + o] : 0.f;
}

void gather_pt(const float *src, const int32_t *perm, int64_t n, int m, int mpad, float *dst, hipStream_t st)
{
    if (n == 0) return;
    hipLaunchKernelGGL(k_gather_pt, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, src, perm, n, m, mpad, dst);
    check_launch(__func__);
}

// out[o] = ||x_o - c_{cell[o * stride]}||^2 (L1: the Manhattan distance;
// float32, it orders the objects inside a cell, nothing more), 16 lanes per
// object.
__global__ void k_centre_dist(const float *__restrict__ X, int dp, int64_t n, const int32_t *__restrict__ cell,
                              int stride, const float *__restrict__ C, float *__restrict__ out, int l1)
{
    const int64_t o = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 4;
    const int sl = threadIdx.x & 15;
    const bool ok = o < n;
    float acc = 0.f;
    if (ok) {
        const float *x = X + (size_t)o * dp;
        const float *c = C + (size_t)cell[o * stride] * dp;
        for (int i = sl; i < dp; i += 16) acc = dev::dterm_rt(l1 != 0, acc, x[i], c[i]);
    }
#pragma unroll
    for (int s = 8; s > 0; s >>= 1) acc += __shfl_xor(acc, s, 16);
    if (ok && sl == 0) out[o] = acc;
}

void centre_dist(const float *X, int dp, int64_t n, const int32_t *cell, int stride, const float *C, float *out,
                 hipStream_t st, bool l1)
{
    if (n == 0) return;
    hipLaunchKernelGGL(k_centre_dist, dim3((unsigned)((n * 16 + 255) / 256)), dim3(256), 0, st, X, dp, n, cell, stride,
                       C, out, l1 ? 1 : 0);
    check_launch(__func__);
}

// Nearest centre of every object by exact float32 distances (the Manhattan
// metric, or rows wider than the bf16 search takes): one thread per object,
// the centres streaming through LDS `per` rows at a time (at most 48 KB);
// the first of equal distances wins.  near[o] = centre number.
__global__ __launch_bounds__(256) void k_nearest_centre(const float *__restrict__ X, int dp, int64_t n,
                                                        const float *__restrict__ C, int K, int per, int l1,
                                                        int32_t *__restrict__ near)
{
    extern __shared__ float s_c[];   // [per][dp]
    const int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const float *x = X + (size_t)(o < n ? o : 0) * dp;
    float best = INFINITY;
    int arg = 0;
    for (int c0 = 0; c0 < K; c0 += per) {
        const int rows = min(per, K - c0);
        __syncthreads();
        for (int i = threadIdx.x; i < rows * dp; i += blockDim.x) s_c[i] = C[(size_t)c0 * dp + i];
        __syncthreads();
        for (int r = 0; r < rows; r++) {
            const float *c = s_c + r * dp;
            float acc = 0.f;
            if (l1)
                for (int i = 0; i < dp; i++) acc = dev::dterm<true>(acc, x[i], c[i]);
            else
                for (int i = 0; i < dp; i++) acc = dev::dterm<false>(acc, x[i], c[i]);
            if (acc < best) {
                best = acc;
                arg = c0 + r;
            }
        }
    }
    if (o < n) near[o] = arg;
}

void nearest_centre(const float *X, int dp, int64_t n, const float *C, int K, bool l1, int32_t *near, hipStream_t st)
{
    if (n == 0) return;
    require((int64_t)dp * sizeof(float) <= ((int64_t)48 << 10), "nearest_centre: rows wider than 48 KB");
    const int per = (int)std::min<int64_t>(16, ((int64_t)48 << 10) / ((int64_t)dp * sizeof(float)));
    hipLaunchKernelGGL(k_nearest_centre, dim3((unsigned)((n + 255) / 256)), dim3(256),
                       (size_t)per * dp * sizeof(float), st, X, dp, n, C, K, per, l1 ? 1 : 0, near);
    check_launch(__func__);
}

// The two sort keys of the leaf order: dist_key[o] = bits of the squared
// distance to the centre (non-negative floats order as their bits), o as the
// value; then, after the stable sort by it, rank_key[p] = chain rank of the
// cell of the object at position p.
__global__ void k_dist_keys(const float *__restrict__ cdist, int64_t n, uint32_t *__restrict__ key,
                            int32_t *__restrict__ val)
{
    const int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (o >= n) return;
    key[o] = __float_as_uint(fmaxf(cdist[o], 0.f));
    val[o] = (int32_t)o;
}

__global__ void k_cell_keys(const int32_t *__restrict__ order, const int32_t *__restrict__ cell, int stride,
                            const int32_t *__restrict__ rank, int64_t n, uint32_t *__restrict__ key)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    key[p] = (uint32_t)rank[cell[(int64_t)order[p] * stride]];
}

void cell_order(const float *cdist, const int32_t *cell, int stride, const int32_t *rank, int n_cells, int64_t n,
                uint32_t *key, int32_t *perm, void *tmp, size_t tmp_bytes, hipStream_t st)
{
    if (n == 0) return;
    const unsigned g = (unsigned)((n + 255) / 256);
    hipLaunchKernelGGL(k_dist_keys, dim3(g), dim3(256), 0, st, cdist, n, key, perm);
    check_launch("cell_order(keys)");
    sort_pairs_u32(key, perm, n, 32, tmp, tmp_bytes, st);
    hipLaunchKernelGGL(k_cell_keys, dim3(g), dim3(256), 0, st, perm, cell, stride, rank, n, key);
    check_launch("cell_order(ranks)");
    int bits = 1;
    while (bits < 31 && ((int64_t)1 << bits) < n_cells) bits++;
    sort_pairs_u32(key, perm, n, bits, tmp, tmp_bytes, st);
}

// Leaf boxes: one workgroup per leaf; thread t takes pivot row t % mpad and
// every (256 / mpad)-th object of the leaf, then the object lanes of each row
// reduce in LDS.  Rows m..mpad-1 span everything when the leaf is not empty
// (they never prune); an empty leaf's box is empty (lo = +inf, hi = -inf).
__global__ __launch_bounds__(256) void k_leaf_boxes(const float *__restrict__ PT, int64_t n, int m, int mpad,
                                                    const int32_t *__restrict__ leaf_first,
                                                    const int32_t *__restrict__ leaf_cnt, int64_t leaf0,
                                                    float *__restrict__ box_aos)
{
    __shared__ float s_lo[256], s_hi[256];
    const int64_t j = blockIdx.x;
    const int i = threadIdx.x % mpad, lane = threadIdx.x / mpad, lanes = 256 / mpad;
    const int64_t a = leaf_first[j];
    const int cnt = leaf_cnt[j];
    float lo = INFINITY, hi = -INFINITY;
    if (i < m && lane < lanes)
        for (int u = lane; u < cnt; u += lanes) {
            const float x = PT[(size_t)i * n + a + u];
            lo = fminf(lo, x);
            hi = fmaxf(hi, x);
        }
    s_lo[threadIdx.x] = lo;
    s_hi[threadIdx.x] = hi;
    __syncthreads();
    if (threadIdx.x < mpad) {
        for (int u = 1; u < lanes; u++) {
            lo = fminf(lo, s_lo[u * mpad + i]);
            hi = fmaxf(hi, s_hi[u * mpad + i]);
        }
        if (i >= m && cnt > 0) {
            lo = -INFINITY;
            hi = INFINITY;
        }
        float *b = box_aos + (size_t)(leaf0 + j) * 2 * mpad;
        b[i] = lo;
        b[mpad + i] = hi;
    }
}

// Nodes [v0, v1) of one level: box = union of the F children's boxes.
__global__ void k_node_boxes(float *__restrict__ box_aos, int64_t v0, int64_t v1, int F, int mpad)
{
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t v = v0 + g / mpad;
    const int i = (int)(g % mpad);
    if (v >= v1) return;
    float lo = INFINITY, hi = -INFINITY;
    for (int c = 0; c < F; c++) {
        const float *b = box_aos + (size_t)(v * F + 1 + c) * 2 * mpad;
        lo = fminf(lo, b[i]);
        hi = fmaxf(hi, b[mpad + i]);
    }
    box_aos[(size_t)v * 2 * mpad + i] = lo;
    box_aos[(size_t)v * 2 * mpad + mpad + i] = hi;
}

__global__ void k_box_soa(const float *__restrict__ box_aos, int64_t n_nodes, int mpad, float *__restrict__ lo,
                          float *__restrict__ hi)
{
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= n_nodes * mpad) return;
    const int64_t v = g / mpad;
    const int i = (int)(g % mpad);
    lo[(size_t)i * n_nodes + v] = box_aos[(size_t)v * 2 * mpad + i];
    hi[(size_t)i * n_nodes + v] = box_aos[(size_t)v * 2 * mpad + mpad + i];
}

void node_boxes(const float *PT, int64_t n, int m, int mpad, const int32_t *leaf_first, const int32_t *leaf_cnt,
                int64_t n_leaves, int64_t leaf0, int64_t n_nodes, int F, int levels, float *box_aos, float *box_lo,
                float *box_hi, hipStream_t st)
{
    require(mpad >= 1 && mpad <= 32 && 256 % mpad == 0, "node_boxes: pivot rows must divide 256");
    hipLaunchKernelGGL(k_leaf_boxes, dim3((unsigned)n_leaves), dim3(256), 0, st, PT, n, m, mpad, leaf_first, leaf_cnt,
                       leaf0, box_aos);
    check_launch("node_boxes(leaves)");
    // levels from the one above the leaves to the root
    int64_t first = leaf0;
    for (int l = levels - 1; l >= 0; l--) {
        const int64_t v0 = (first - 1) / F, v1 = first;   // this level: [v0, first)
        const int64_t threads = (v1 - v0) * mpad;
        hipLaunchKernelGGL(k_node_boxes, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, st, box_aos, v0, v1,
                           F, mpad);
        check_launch("node_boxes(level)");
        first = v0;
    }
    const int64_t threads = n_nodes * mpad;
    hipLaunchKernelGGL(k_box_soa, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, st, box_aos, n_nodes, mpad,
                       box_lo, box_hi);
    check_launch("node_boxes(soa)");
}

// One wave per slab: the largest rounding error and norm over its rows (with
// a relative margin for the rounding of the summaries themselves), and the
// first and last leaf overlapping it (leaf_first ascending).
__global__ void k_slab_summary(const float *__restrict__ xn, const float *__restrict__ xe, int64_t n,
                               const int32_t *__restrict__ leaf_first, int64_t n_leaves, int64_t n_slabs,
                               float *__restrict__ emax, float *__restrict__ nmax, int32_t *__restrict__ sl,
                               int32_t *__restrict__ sh)
{
    const int64_t s = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int lane = threadIdx.x & 63;
    if (s >= n_slabs) return;   // whole waves leave together
    const int64_t a = s * kSlab, b = min<int64_t>(n, a + kSlab);
    float e = 0.f, r = 0.f;
    for (int64_t p = a + lane; p < b; p += 64) {
        e = fmaxf(e, xe[p]);
        r = fmaxf(r, sqrtf(xn[p]));
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        e = fmaxf(e, __shfl_xor(e, o, 64));
        r = fmaxf(r, __shfl_xor(r, o, 64));
    }
    if (lane == 0) {
        emax[s] = e * 1.0001f + 1e-30f;
        nmax[s] = r * 1.0001f;
        // last leaf whose first position is <= x, for x = a and x = b - 1
        auto leaf_at = [&](int64_t x) {
            int64_t lo = 0, hi = n_leaves;   // leaf_first[lo - 1] <= x < leaf_first[hi]
            while (lo < hi) {
                const int64_t mid = (lo + hi) >> 1;
                if (leaf_first[mid] <= x) lo = mid + 1;
                else hi = mid;
            }
            return lo - 1;
        };
        sl[s] = (int32_t)max<int64_t>(0, leaf_at(a));
        sh[s] = (int32_t)max<int64_t>(0, leaf_at(max<int64_t>(a, b - 1)));
    }
}

void slab_summary(const float *xn, const float *xe, int64_t n, const int32_t *leaf_first, int64_t n_leaves,
                  int64_t n_slabs, float *emax, float *nmax, int32_t *sl, int32_t *sh, hipStream_t st)
{
    if (n_slabs == 0) return;
    hipLaunchKernelGGL(k_slab_summary, dim3((unsigned)((n_slabs * 64 + 255) / 256)), dim3(256), 0, st, xn, xe, n,
                       leaf_first, n_leaves, n_slabs, emax, nmax, sl, sh);
    check_launch(__func__);
}

// cen[j][c] = mean of coordinate c over leaf j's objects, summed in double in
// position order (one thread per coordinate).
__global__ __launch_bounds__(256) void k_leaf_centroid(const float *__restrict__ X32, int dp, int dim,
                                                       const int32_t *__restrict__ leaf_first,
                                                       const int32_t *__restrict__ leaf_cnt,
                                                       double *__restrict__ cen)
{
    const int64_t j = blockIdx.x;
    const int64_t a = leaf_first[j];
    const int cnt = leaf_cnt[j];
    for (int c = threadIdx.x; c < dim; c += blockDim.x) {
        double s = 0.0;
        for (int u = 0; u < cnt; u++) s += X32[(size_t)(a + u) * dp + c];
        cen[(size_t)j * dim + c] = cnt > 0 ? s / (double)cnt : 0.0;
    }
}

// Per leaf j < lpad: the object nearest the centroid (squared distance in
// double, coordinates in order; the first position wins ties), its row into
// PL32 and the largest distance from it to the leaf's objects, in double,
// widened by a relative 1e-6 so that the float bounds the true value (l1:
// Manhattan distances throughout).  An
// empty leaf (or j >= n_leaves) gets a zero row and R = -inf.
__global__ __launch_bounds__(256) void k_leaf_pivot(const float *__restrict__ X32, int dp, int dim,
                                                    const int32_t *__restrict__ leaf_first,
                                                    const int32_t *__restrict__ leaf_cnt, int64_t n_leaves,
                                                    const double *__restrict__ cen, float *__restrict__ PL32,
                                                    float *__restrict__ leafR, int l1)
{
    __shared__ double s_v[256];
    __shared__ int32_t s_p[256];
    const int64_t j = blockIdx.x;
    const int cnt = j < n_leaves ? leaf_cnt[j] : 0;
    float *row = PL32 + (size_t)j * dp;
    if (cnt == 0) {
        for (int c = threadIdx.x; c < dp; c += blockDim.x) row[c] = 0.f;
        if (threadIdx.x == 0) leafR[j] = -INFINITY;
        return;
    }
    const int64_t a = leaf_first[j];
    const double *ce = cen + (size_t)j * dim;
    double bv = INFINITY;
    int32_t bp = INT32_MAX;
    for (int u = threadIdx.x; u < cnt; u += blockDim.x) {
        const float *x = X32 + (size_t)(a + u) * dp;
        double s2 = 0.0;
        for (int c = 0; c < dim; c++) {
            const double df = (double)x[c] - ce[c];
            s2 += l1 ? fabs(df) : df * df;
        }
        if (s2 < bv) {   // u ascends within a thread: the first minimum stays
            bv = s2;
            bp = u;
        }
    }
    s_v[threadIdx.x] = bv;
    s_p[threadIdx.x] = bp;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            const double v2 = s_v[threadIdx.x + w];
            const int32_t p2 = s_p[threadIdx.x + w];
            if (v2 < s_v[threadIdx.x] || (v2 == s_v[threadIdx.x] && p2 < s_p[threadIdx.x])) {
                s_v[threadIdx.x] = v2;
                s_p[threadIdx.x] = p2;
            }
        }
        __syncthreads();
    }
    const int64_t best = a + s_p[0];
    __syncthreads();
    const float *y = X32 + (size_t)best * dp;
    double rmax = 0.0;
    for (int u = threadIdx.x; u < cnt; u += blockDim.x) {
        const float *x = X32 + (size_t)(a + u) * dp;
        double s2 = 0.0;
        for (int c = 0; c < dim; c++) {
            const double df = (double)x[c] - (double)y[c];
            s2 += l1 ? fabs(df) : df * df;
        }
        rmax = fmax(rmax, l1 ? s2 : sqrt(s2));
    }
    s_v[threadIdx.x] = rmax;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) s_v[threadIdx.x] = fmax(s_v[threadIdx.x], s_v[threadIdx.x + w]);
        __syncthreads();
    }
    for (int c = threadIdx.x; c < dp; c += blockDim.x) row[c] = y[c];
    if (threadIdx.x == 0) leafR[j] = (float)(s_v[0] * (1.0 + 1e-6)) + 1e-30f;
}

// pln[j] = +inf for leaves that hold no object (never a nearest leaf).
__global__ void k_mark_empty(const int32_t *__restrict__ leaf_cnt, int64_t n_leaves, int64_t lpad,
                             float *__restrict__ pln)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j < lpad && (j >= n_leaves || leaf_cnt[j] == 0)) pln[j] = INFINITY;
}

void leaf_pivots(const float *X32, int dp, int dim, const int32_t *leaf_first, const int32_t *leaf_cnt,
                 int64_t n_leaves, int64_t lpad, double *cen, float *PL32, float *leafR, hipStream_t st, bool l1)
{
    hipLaunchKernelGGL(k_leaf_centroid, dim3((unsigned)n_leaves), dim3(256), 0, st, X32, dp, dim, leaf_first, leaf_cnt,
                       cen);
    check_launch("leaf_pivots(centroid)");
    hipLaunchKernelGGL(k_leaf_pivot, dim3((unsigned)lpad), dim3(256), 0, st, X32, dp, dim, leaf_first, leaf_cnt,
                       n_leaves, cen, PL32, leafR, l1 ? 1 : 0);
    check_launch("leaf_pivots(pivot)");
}

void mark_empty(const int32_t *leaf_cnt, int64_t n_leaves, int64_t lpad, float *pln, hipStream_t st)
{
    hipLaunchKernelGGL(k_mark_empty, dim3((unsigned)((lpad + 255) / 256)), dim3(256), 0, st, leaf_cnt, n_leaves, lpad,
                       pln);
    check_launch(__func__);
}

// *out = max(*out, max_i x[i]) for non-negative floats (their bits order as
// the values); *out must start at 0.
__global__ void k_max_f32(const float *__restrict__ x, int64_t n, uint32_t *__restrict__ out)
{
    float v = 0.f;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        v = fmaxf(v, x[i]);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
    if ((threadIdx.x & 63) == 0) atomicMax(out, __float_as_uint(v));
}

void max_f32(const float *x, int64_t n, uint32_t *out, hipStream_t st)
{
    if (n == 0) return;
    const int64_t blocks = std::min<int64_t>(1024, (n + 255) / 256);
    hipLaunchKernelGGL(k_max_f32, dim3((unsigned)blocks), dim3(256), 0, st, x, n, out);
    check_launch(__func__);
}

}  // namespace k
}  // namespace gts
