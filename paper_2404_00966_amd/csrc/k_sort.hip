// Query order by home (leaf or cell) on the device: a stable radix sort of
// the home keys (rocPRIM) carrying the query index, so the permutation is the
// same on every run and no host round trip sits between the search for the
// homes and the first kernel that reads the queries in the new order.
#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/iterator/counting_iterator.hpp>

#include "kernels.h"

namespace gts {
namespace k {

__global__ void k_home_keys(const int32_t *__restrict__ home, int stride, int64_t nq, uint32_t *__restrict__ key)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < nq) key[q] = (uint32_t)home[q * stride];
}

static int key_bits(int64_t n_keys)
{
    int b = 1;
    while (b < 31 && ((int64_t)1 << b) < n_keys) b++;
    return b;
}

size_t home_sort_bytes(int64_t nq, int64_t n_keys)
{
    size_t bytes = 0;
    const uint32_t *kin = nullptr;
    uint32_t *kout = nullptr;
    int32_t *vout = nullptr;
    const hipError_t e = rocprim::radix_sort_pairs(nullptr, bytes, kin, kout, rocprim::counting_iterator<int32_t>(0),
                                                   vout, (size_t)nq, 0u, (unsigned)key_bits(n_keys));
    require(e == hipSuccess, "home_sort_bytes: rocprim size query failed");
    return bytes;
}

void home_sort(const int32_t *home, int stride, int64_t nq, int64_t n_keys, uint32_t *keys, uint32_t *keys_sorted,
               int32_t *perm, void *tmp, size_t tmp_bytes, hipStream_t st)
{
    if (nq == 0) return;
    require(n_keys > 0 && n_keys < ((int64_t)1 << 31) && stride >= 1, "home_sort: key range out of bounds");
    hipLaunchKernelGGL(k_home_keys, dim3((unsigned)((nq + 255) / 256)), dim3(256), 0, st, home, stride, nq, keys);
    check_launch(__func__);
    size_t bytes = tmp_bytes;
    const hipError_t e = rocprim::radix_sort_pairs(tmp, bytes, keys, keys_sorted,
                                                   rocprim::counting_iterator<int32_t>(0), perm, (size_t)nq, 0u,
                                                   (unsigned)key_bits(n_keys), st);
    require(e == hipSuccess, "home_sort: rocprim radix sort failed");
}

}  // namespace k
}  // namespace gts
