// Selection of the exchange step (Sec. 2.2): the k_eff first candidates of a
// list in the order (key, then SplitMix64 hash of the cell index).  The keys
// kernel stores the solid list's keys bit-complemented, so ascending order
// here is descending key order there.  The hash is a bijection of the index,
// so the pair (key, hash) orders a list totally.  Two stable LSD radix sorts
// (library primitive), by hash and then by key, leave the list in exactly
// that order.
#include <hip/hip_runtime.h>

#include <hipcub/hipcub.hpp>

#include "lbm_internal.h"

namespace lbm {

namespace {

__global__ void iota_kernel(uint32_t *p, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = (uint32_t)i;
}

// key2[j] = key[perm[j]].
__global__ void gather_keys_kernel(const uint64_t *key, const uint32_t *perm, int64_t n,
                                   uint64_t *key2) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j < n) key2[j] = key[perm[j]];
}

__global__ void take_kernel(const int32_t *idx, const uint32_t *perm, int64_t k_eff,
                            int32_t *sel) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j < k_eff) sel[j] = idx[perm[j]];
}

size_t align256(size_t b) { return (b + 255) / 256 * 256; }

struct Layout {
    size_t hash_out, perm_a, perm_b, key2, key2_out, cub, cub_bytes, total;
};

Layout layout(int64_t cap) {
    size_t cub_a = 0, cub_b = 0;
    (void)hipcub::DeviceRadixSort::SortPairs(nullptr, cub_a, (const uint64_t *)nullptr,
                                             (uint64_t *)nullptr, (const uint32_t *)nullptr,
                                             (uint32_t *)nullptr, (int)cap);
    cub_b = cub_a;
    Layout L;
    size_t o = 0;
    L.hash_out = o;
    o += align256((size_t)cap * 8);
    L.perm_a = o;
    o += align256((size_t)cap * 4);
    L.perm_b = o;
    o += align256((size_t)cap * 4);
    L.key2 = o;
    o += align256((size_t)cap * 8);
    L.key2_out = o;
    o += align256((size_t)cap * 8);
    L.cub = o;
    L.cub_bytes = align256(std::max(cub_a, cub_b));
    o += L.cub_bytes;
    L.total = o;
    return L;
}

}  // namespace

size_t select_scratch_bytes(int64_t cap) { return layout(std::max<int64_t>(cap, 1)).total; }

hipError_t launch_select(const uint64_t *key, const uint64_t *hash, const int32_t *idx,
                         int64_t count, int64_t k_eff, int32_t *sel,
                         void *scratch, int64_t cap, hipStream_t s) {
    if (count <= 0 || k_eff <= 0) return hipSuccess;
    if (count > cap || k_eff > count || count > INT32_MAX) return hipErrorInvalidValue;
    const Layout L = layout(cap);
    unsigned char *b = static_cast<unsigned char *>(scratch);
    uint64_t *hash_out = reinterpret_cast<uint64_t *>(b + L.hash_out);
    uint32_t *pa = reinterpret_cast<uint32_t *>(b + L.perm_a);
    uint32_t *pb = reinterpret_cast<uint32_t *>(b + L.perm_b);
    uint64_t *key2 = reinterpret_cast<uint64_t *>(b + L.key2);
    uint64_t *key2_out = reinterpret_cast<uint64_t *>(b + L.key2_out);
    void *cub = b + L.cub;
    const unsigned g = (unsigned)((count + 255) / 256);
    hipLaunchKernelGGL(iota_kernel, dim3(g), dim3(256), 0, s, pa, count);
    size_t tb = L.cub_bytes;
    hipError_t e = hipcub::DeviceRadixSort::SortPairs(cub, tb, hash, hash_out, pa, pb,
                                                      (int)count, 0, 64, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(gather_keys_kernel, dim3(g), dim3(256), 0, s, key, pb, count, key2);
    tb = L.cub_bytes;
    e = hipcub::DeviceRadixSort::SortPairs(cub, tb, key2, key2_out, pb, pa, (int)count, 0, 64,
                                           s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(take_kernel, dim3((unsigned)((k_eff + 255) / 256)), dim3(256), 0, s, idx,
                       pa, k_eff, sel);
    return hipGetLastError();
}

}  // namespace lbm
