// Selection of the exchange step (Sec. 2.2): the k_eff first candidates of
// each list in the order (key, then SplitMix64 hash of the cell index).  The
// keys kernel stores the solid list's keys bit-complemented, so ascending
// order here is descending key order there.  The hash is a bijection of the
// index, so the pair (key, hash) orders a list totally.
//
// Both lists are sorted in one pass: fluid keys are images of doubles >= +0
// (top bit clear) and complemented solid keys have the top bit set, so in
// the concatenated list every fluid candidate sorts before every solid one
// and each part keeps its own order.  Two stable LSD radix sorts (library
// primitive), by hash and then by key, leave the list in exactly that order.
#include <hip/hip_runtime.h>

#include <hipcub/hipcub.hpp>

#include "lbm_internal.h"

namespace lbm {

namespace {

// Concatenate the two lists: entries [0, nf) from the fluid list, then
// [nf, nf + ns) from the solid list; perm = identity.
__global__ void pack_kernel(const uint64_t *kf, const uint64_t *hf, const int32_t *if_,
                            int64_t nf, const uint64_t *ks, const uint64_t *hs,
                            const int32_t *is, int64_t ns, uint64_t *key, uint64_t *hash,
                            int32_t *idx, uint32_t *perm) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= nf + ns) return;
    const bool f = j < nf;
    const int64_t s = f ? j : j - nf;
    key[j] = f ? kf[s] : ks[s];
    hash[j] = f ? hf[s] : hs[s];
    idx[j] = f ? if_[s] : is[s];
    perm[j] = (uint32_t)j;
}

// key2[j] = key[perm[j]].
__global__ void gather_keys_kernel(const uint64_t *key, const uint32_t *perm, int64_t n,
                                   uint64_t *key2) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j < n) key2[j] = key[perm[j]];
}

// The first k_eff of each part of the sorted list.
__global__ void take_kernel(const int32_t *idx, const uint32_t *perm, int64_t nf,
                            int64_t k_eff, int32_t *sel_f, int32_t *sel_s) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= k_eff) return;
    sel_f[j] = idx[perm[j]];
    sel_s[j] = idx[perm[nf + j]];
}

size_t align256(size_t b) { return (b + 255) / 256 * 256; }

struct Layout {
    size_t key, hash, idx, hash_out, perm_a, perm_b, key2, key2_out, cub, cub_bytes, total;
};

// Scratch for two lists of at most cap entries each.
Layout layout(int64_t cap) {
    const int64_t n = 2 * cap;
    size_t cub_bytes = 0;
    (void)hipcub::DeviceRadixSort::SortPairs(nullptr, cub_bytes, (const uint64_t *)nullptr,
                                             (uint64_t *)nullptr, (const uint32_t *)nullptr,
                                             (uint32_t *)nullptr, (int)n);
    Layout L;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o += align256(bytes);
        return at;
    };
    L.key = take((size_t)n * 8);
    L.hash = take((size_t)n * 8);
    L.idx = take((size_t)n * 4);
    L.hash_out = take((size_t)n * 8);
    L.perm_a = take((size_t)n * 4);
    L.perm_b = take((size_t)n * 4);
    L.key2 = take((size_t)n * 8);
    L.key2_out = take((size_t)n * 8);
    L.cub_bytes = align256(cub_bytes);
    L.cub = take(L.cub_bytes);
    L.total = o;
    return L;
}

}  // namespace

size_t select_scratch_bytes(int64_t cap) { return layout(std::max<int64_t>(cap, 1)).total; }

hipError_t launch_select_pair(const uint64_t *kf, const uint64_t *hf, const int32_t *if_,
                              int64_t nf, const uint64_t *ks, const uint64_t *hs,
                              const int32_t *is, int64_t ns, int64_t k_eff, int32_t *sel_f,
                              int32_t *sel_s, void *scratch, int64_t cap, hipStream_t s) {
    if (k_eff <= 0) return hipSuccess;
    if (nf > cap || ns > cap || k_eff > nf || k_eff > ns || nf + ns > INT32_MAX)
        return hipErrorInvalidValue;
    const Layout L = layout(cap);
    const int64_t n = nf + ns;
    unsigned char *b = static_cast<unsigned char *>(scratch);
    uint64_t *key = reinterpret_cast<uint64_t *>(b + L.key);
    uint64_t *hash = reinterpret_cast<uint64_t *>(b + L.hash);
    int32_t *idx = reinterpret_cast<int32_t *>(b + L.idx);
    uint64_t *hash_out = reinterpret_cast<uint64_t *>(b + L.hash_out);
    uint32_t *pa = reinterpret_cast<uint32_t *>(b + L.perm_a);
    uint32_t *pb = reinterpret_cast<uint32_t *>(b + L.perm_b);
    uint64_t *key2 = reinterpret_cast<uint64_t *>(b + L.key2);
    uint64_t *key2_out = reinterpret_cast<uint64_t *>(b + L.key2_out);
    void *cub = b + L.cub;
    const unsigned g = (unsigned)((n + 255) / 256);
    hipLaunchKernelGGL(pack_kernel, dim3(g), dim3(256), 0, s, kf, hf, if_, nf, ks, hs, is, ns,
                       key, hash, idx, pa);
    size_t tb = L.cub_bytes;
    hipError_t e = hipcub::DeviceRadixSort::SortPairs(cub, tb, hash, hash_out, pa, pb, (int)n,
                                                      0, 64, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(gather_keys_kernel, dim3(g), dim3(256), 0, s, key, pb, n, key2);
    tb = L.cub_bytes;
    e = hipcub::DeviceRadixSort::SortPairs(cub, tb, key2, key2_out, pb, pa, (int)n, 0, 64, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(take_kernel, dim3((unsigned)((k_eff + 255) / 256)), dim3(256), 0, s, idx,
                       pa, nf, k_eff, sel_f, sel_s);
    return hipGetLastError();
}

}  // namespace lbm
