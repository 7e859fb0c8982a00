// Selection of the exchange step (Sec. 2.2, Eqs. 5-6; Sec. 2.3 step 3): the
// k_eff first candidates of each list in the order (key, then SplitMix64 hash
// of the cell index), written as cell indices in that order.  The keys kernel
// stores the solid list's keys bit-complemented, so ascending order here is
// descending key order there.  The hash is a bijection of the cell index, so
// the 128-bit composite (key, hash) of a list's candidates is unique and
// orders the list totally.
//
// Integer work only, in four kernels per chunk of at most kChunk ranks (one
// chunk unless k_eff is very large):
//   narrow   one workgroup per list finds the composite of rank r (the last
//            rank of the chunk) exactly: a most-significant-digit radix
//            select over the 16 bytes of the composite, one LDS histogram
//            per byte of the bucket holding rank r, until that bucket holds a
//            single candidate;
//   compact  every candidate whose composite lies in (previous chunk's
//            threshold, this chunk's threshold] is copied to a dense chunk
//            list (one atomic per wave);
//   rank     each chunk entry counts the entries below it (LDS tiles, a 2-D
//            grid; partial counts added atomically);
//   scatter  entry i goes to output position chunk base + rank i.
// The result is fixed by the candidates alone, whatever the scheduling.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "lbm_internal.h"

namespace lbm {

namespace {

constexpr int64_t kChunk = 32768;  // ranks per chunk (ranking is quadratic in it)
constexpr int kNarrowThreads = 1024;
constexpr int kRankRows = 256, kRankCols = 1024;

struct Cand {
    const uint64_t *key, *hash;
    const int32_t *idx;
    int64_t n;
};

// Per-list selection state on the device.
struct SelState {
    uint64_t thr_key[2], thr_hash[2];  // composite of the current chunk's last rank
    uint64_t lo_key[2], lo_hash[2];    // the previous chunk's threshold
    unsigned long long count[2];       // entries compacted for the current chunk
    int error;
};

__device__ __forceinline__ bool less128(uint64_t ak, uint64_t ah, uint64_t bk, uint64_t bh) {
    return ak < bk || (ak == bk && ah < bh);
}

// Byte d (0 = most significant) of the composite key:hash.
__device__ __forceinline__ uint32_t digit(uint64_t k, uint64_t h, int d) {
    const uint64_t w = d < 8 ? k : h;
    return (uint32_t)(w >> (56 - 8 * (d & 7))) & 0xffu;
}

// Block b finds the composite of rank r of list b.
__global__ __launch_bounds__(kNarrowThreads) void narrow_kernel(Cand c0, Cand c1, int64_t r,
                                                                SelState *st) {
    const Cand c = blockIdx.x == 0 ? c0 : c1;
    const int b = blockIdx.x, tid = threadIdx.x;
    __shared__ unsigned hist[256];
    __shared__ int64_t witness[256];
    __shared__ int64_t s_rank, s_count, s_wit;
    __shared__ uint32_t s_digit;
    uint64_t pk = 0, ph = 0, mk = 0, mh = 0;  // digits fixed so far, and their mask
    int64_t rr = r;                            // rank within the current bucket
    int d = 0;
    for (; d < 16; ++d) {
        if (tid < 256) hist[tid] = 0u;
        if (tid == 0) {
            s_count = 0;
            s_wit = -1;
        }
        __syncthreads();
        for (int64_t i = tid; i < c.n; i += kNarrowThreads) {
            const uint64_t k = c.key[i], h = c.hash[i];
            if (((k ^ pk) & mk) == 0 && ((h ^ ph) & mh) == 0) {
                const uint32_t v = digit(k, h, d);
                atomicAdd(&hist[v], 1u);
                witness[v] = i;  // read only when the bin holds one candidate
            }
        }
        __syncthreads();
        if (tid < 64) {
            // lane l owns bins 4l..4l+3; exclusive prefix over the lanes
            unsigned hv[4], s = 0;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                hv[q] = hist[4 * tid + q];
                s += hv[q];
            }
            int64_t incl = s;
#pragma unroll
            for (int off = 1; off < 64; off <<= 1) {
                const int64_t o = __shfl_up(incl, off, 64);
                if (tid >= off) incl += o;
            }
            int64_t base = incl - s;
            if (base <= rr && rr < incl) {
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    if (base <= rr && rr < base + (int64_t)hv[q]) {
                        s_digit = 4u * tid + q;
                        s_rank = rr - base;
                        s_count = hv[q];
                        s_wit = witness[4 * tid + q];
                    }
                    base += hv[q];
                }
            }
        }
        __syncthreads();
        const uint32_t v = s_digit;
        rr = s_rank;
        const int64_t cnt = s_count;
        const int64_t wit = s_wit;
        const int sh = 56 - 8 * (d & 7);
        if (d < 8) {
            pk |= (uint64_t)v << sh;
            mk |= 0xffull << sh;
        } else {
            ph |= (uint64_t)v << sh;
            mh |= 0xffull << sh;
        }
        if (cnt == 0 || (cnt == 1 && (wit < 0 || wit >= c.n))) {
            if (tid == 0) st->error |= 16;  // rank outside the list: unreachable
            return;
        }
        if (cnt == 1) {
            if (tid == 0) {
                st->thr_key[b] = c.key[wit];
                st->thr_hash[b] = c.hash[wit];
                st->count[b] = 0ull;
            }
            return;
        }
        __syncthreads();  // the shared results are read before the next pass writes them
    }
    if (tid == 0) st->error = 1;  // composites are unique: unreachable for valid input
}

// Candidates of list blockIdx.y with composite in (lo, thr] (lo only when
// has_lo) into the dense chunk lists.
__global__ __launch_bounds__(256) void compact_kernel(Cand c0, Cand c1, int has_lo,
                                                      SelState *st, uint64_t *ck,
                                                      uint64_t *chh, int32_t *ci,
                                                      int64_t cap) {
    const int b = blockIdx.y;
    const Cand c = b == 0 ? c0 : c1;
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    bool take = false;
    uint64_t k = 0, h = 0;
    if (i < c.n) {
        k = c.key[i];
        h = c.hash[i];
        take = !less128(st->thr_key[b], st->thr_hash[b], k, h) &&
               (!has_lo || less128(st->lo_key[b], st->lo_hash[b], k, h));
    }
    const int lane = threadIdx.x & 63;
    const uint64_t m = __ballot(take);
    unsigned long long base = 0;
    if (lane == 0 && m) base = atomicAdd(&st->count[b], (unsigned long long)__popcll(m));
    base = __shfl(base, 0, 64);
    if (!take) return;
    const unsigned long long slot = base + __popcll(m & ((1ull << lane) - 1ull));
    if ((int64_t)slot >= cap) {
        atomicOr(&st->error, 2);
        return;
    }
    ck[b * cap + slot] = k;
    chh[b * cap + slot] = h;
    ci[b * cap + slot] = c.idx[i];
}

// rank[i] += number of chunk entries j below entry i, for the column tile
// blockIdx.y of list blockIdx.z.
__global__ __launch_bounds__(kRankRows) void rank_kernel(const uint64_t *ck, const uint64_t *chh,
                                                         int64_t m, int64_t cap,
                                                         uint32_t *rank) {
    __shared__ uint64_t tk[kRankCols], th[kRankCols];
    const int b = blockIdx.z;
    const uint64_t *K = ck + b * cap, *H = chh + b * cap;
    const int64_t i = (int64_t)blockIdx.x * kRankRows + threadIdx.x;
    const int64_t j0 = (int64_t)blockIdx.y * kRankCols;
    const int64_t nj = std::min<int64_t>(kRankCols, m - j0);
    for (int t = threadIdx.x; t < nj; t += kRankRows) {
        tk[t] = K[j0 + t];
        th[t] = H[j0 + t];
    }
    __syncthreads();
    if (i >= m) return;
    const uint64_t k = K[i], h = H[i];
    uint32_t cnt = 0;
    for (int t = 0; t < nj; ++t) cnt += less128(tk[t], th[t], k, h) ? 1u : 0u;
    if (cnt) atomicAdd(&rank[b * cap + i], cnt);
}

// Output position base + rank of each chunk entry; a chunk whose size or
// ranks disagree with the selection is flagged.
__global__ __launch_bounds__(256) void scatter_kernel(const int32_t *ci, const uint32_t *rank,
                                                      int64_t m, int64_t cap, int64_t base,
                                                      SelState *st, int32_t *sel_f,
                                                      int32_t *sel_s) {
    const int b = blockIdx.y;
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i == 0 && st->count[b] != (unsigned long long)m) atomicOr(&st->error, 4);
    if (i >= m) return;
    const uint32_t r = rank[b * cap + i];
    if ((int64_t)r >= m) {
        atomicOr(&st->error, 8);
        return;
    }
    (b == 0 ? sel_f : sel_s)[base + r] = ci[b * cap + i];
}

// The chunk's threshold becomes the next chunk's lower bound.
__global__ void advance_kernel(SelState *st) {
    const int b = threadIdx.x;
    if (b < 2) {
        st->lo_key[b] = st->thr_key[b];
        st->lo_hash[b] = st->thr_hash[b];
    }
}

__global__ void init_kernel(SelState *st) {
    if (threadIdx.x == 0) {
        st->error = 0;
        st->count[0] = st->count[1] = 0ull;
    }
}

// The state's error word, shifted above the keys kernel's, into the caller's
// flag.
__global__ void report_kernel(const SelState *st, int *err) {
    if (threadIdx.x == 0 && st->error) atomicOr(err, st->error << 8);
}

__global__ void zero_u32_kernel(uint32_t *p, int64_t count) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}

size_t align256(size_t b) { return (b + 255) / 256 * 256; }

// Scratch: the state, then per list and chunk entry a key, a hash, an index
// and a rank.
struct Layout {
    size_t state, key, hash, idx, rank, total;
    int64_t cap;
};

Layout layout(int64_t k_max) {
    Layout L;
    L.cap = std::max<int64_t>(1, std::min<int64_t>(k_max, kChunk));
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o += align256(bytes);
        return at;
    };
    L.state = take(sizeof(SelState));
    L.key = take((size_t)2 * L.cap * 8);
    L.hash = take((size_t)2 * L.cap * 8);
    L.idx = take((size_t)2 * L.cap * 4);
    L.rank = take((size_t)2 * L.cap * 4);
    L.total = o;
    return L;
}

}  // namespace

size_t select_scratch_bytes(int64_t k_max) { return layout(k_max).total; }

hipError_t launch_select_pair(const uint64_t *kf, const uint64_t *hf, const int32_t *if_,
                              int64_t nf, const uint64_t *ks, const uint64_t *hs,
                              const int32_t *is, int64_t ns, int64_t k_eff, int32_t *sel_f,
                              int32_t *sel_s, void *scratch, int64_t k_max, int *error,
                              hipStream_t s) {
    if (k_eff <= 0) return hipSuccess;
    if (k_eff > nf || k_eff > ns || k_eff > k_max || nf > INT32_MAX || ns > INT32_MAX)
        return hipErrorInvalidValue;
    const Layout L = layout(k_max);
    unsigned char *p = static_cast<unsigned char *>(scratch);
    SelState *st = reinterpret_cast<SelState *>(p + L.state);
    uint64_t *ck = reinterpret_cast<uint64_t *>(p + L.key);
    uint64_t *chh = reinterpret_cast<uint64_t *>(p + L.hash);
    int32_t *ci = reinterpret_cast<int32_t *>(p + L.idx);
    uint32_t *rank = reinterpret_cast<uint32_t *>(p + L.rank);
    const Cand c0{kf, hf, if_, nf}, c1{ks, hs, is, ns};
    const int64_t nmax = std::max(nf, ns);
    hipLaunchKernelGGL(init_kernel, dim3(1), dim3(64), 0, s, st);
    for (int64_t lo = 0; lo < k_eff; lo += L.cap) {
        const int64_t hi = std::min(k_eff, lo + L.cap), m = hi - lo;
        hipLaunchKernelGGL(narrow_kernel, dim3(2), dim3(kNarrowThreads), 0, s, c0, c1, hi - 1,
                           st);
        hipLaunchKernelGGL(zero_u32_kernel, dim3((unsigned)std::min<int64_t>(1024, (2 * m + 255) / 256)),
                           dim3(256), 0, s, rank, 2 * L.cap);
        hipLaunchKernelGGL(compact_kernel, dim3((unsigned)((nmax + 255) / 256), 2), dim3(256), 0,
                           s, c0, c1, lo > 0 ? 1 : 0, st, ck, chh, ci, L.cap);
        hipLaunchKernelGGL(rank_kernel,
                           dim3((unsigned)((m + kRankRows - 1) / kRankRows),
                                (unsigned)((m + kRankCols - 1) / kRankCols), 2),
                           dim3(kRankRows), 0, s, ck, chh, m, L.cap, rank);
        hipLaunchKernelGGL(scatter_kernel, dim3((unsigned)((m + 255) / 256), 2), dim3(256), 0, s,
                           ci, rank, m, L.cap, lo, st, sel_f, sel_s);
        if (hi < k_eff) hipLaunchKernelGGL(advance_kernel, dim3(1), dim3(64), 0, s, st);
    }
    hipLaunchKernelGGL(report_kernel, dim3(1), dim3(64), 0, s, st, error);
    return hipGetLastError();
}

}  // namespace lbm
