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
#include <cstdlib>

#include "lbm_internal.h"

namespace lbm {

namespace {

constexpr int64_t kChunk = 32768;  // ranks per chunk (ranking is quadratic in it)
constexpr int kNarrowThreads = 1024;
constexpr int kNarrowCached = 16;  // candidates per thread kept in registers
constexpr int kRankRows = 256, kRankCols = 128;
constexpr int kPassThreads = 256, kMaxPassBlocks = 512;
// Multi-block passes queued for a long list (each launch costs a few
// microseconds even when the select is already done); what they leave is
// finished by one workgroup per list.  On the distributors' lists (45k-150k
// candidates) 2 to 16 queued passes measured the same within noise.
constexpr int kPassLaunches = 4;

struct Cand {
    const uint64_t *key, *hash;
    const int32_t *idx;
    int64_t n;
};

struct Narrow {
    uint64_t pk, ph, mk, mh;  // digits fixed so far (key, hash) and their masks
    int64_t rr;               // rank within the current bucket
    int d;                    // next digit
    int done;                 // the threshold is known
};

// Per-list selection state on the device.
struct SelState {
    uint64_t thr_key[2], thr_hash[2];  // composite of the current chunk's last rank
    uint64_t lo_key[2], lo_hash[2];    // the previous chunk's threshold
    unsigned long long count[2];       // entries compacted for the current chunk
    int error;
    // multi-block narrowing, per list: the select's state, the pass's
    // finished-block count, and the pass's histogram (count, one witness and
    // the key range per bin)
    Narrow nar[2];
    unsigned ticket[2];
    unsigned hist[2][256];
    int64_t wit[2][256];
    uint64_t kmin[2][256], kmax[2][256];
};

__device__ __forceinline__ bool less128(uint64_t ak, uint64_t ah, uint64_t bk, uint64_t bh) {
    return ak < bk || (ak == bk && ah < bh);
}

// Byte d (0 = most significant) of the composite key:hash.
__device__ __forceinline__ uint32_t digit(uint64_t k, uint64_t h, int d) {
    const uint64_t w = d < 8 ? k : h;
    return (uint32_t)(w >> (56 - 8 * (d & 7))) & 0xffu;
}

// Radix select of the composite of rank r, one byte (digit) at a time: the
// candidates sharing the fixed digits form the current bucket; the histogram
// of their next digit gives the bin holding rank r, which becomes the bucket.
// Besides the count, each bin records one candidate (meaningful when it is
// alone) and, while the digit is a key byte, the smallest and largest key of
// its candidates: all keys of the new bucket then share the leading bytes of
// those two, so the select jumps past the bytes they have in common (past
// the whole key when they are equal, e.g. keys tied at zero).

__device__ __forceinline__ uint64_t top_bytes(int j) { return j <= 0 ? 0ull : ~0ull << (64 - 8 * j); }

// Histogram contribution of one candidate (all lanes of the wave call this
// together).  A wave whose matching candidates share the digit (the usual
// case in the leading bytes) updates the bin once.
template <class AddCount, class SetWitness, class MinMax>
__device__ __forceinline__ void bin_candidate(bool match, uint64_t k, uint64_t h, int d, int64_t i,
                                              int lane, AddCount add, SetWitness wit,
                                              MinMax minmax) {
    const uint32_t v = digit(k, h, d);
    const uint64_t mm = __ballot(match);
    if (mm == 0) return;
    const int first = __ffsll((long long)mm) - 1;
    const uint32_t v0 = __shfl(v, first, 64);
    if (__ballot(match && v == v0) == mm) {
        uint64_t kn = match ? k : ~0ull, kx = match ? k : 0ull;
        if (d < 8) {
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) {
                kn = min(kn, (uint64_t)__shfl_xor(kn, off, 64));
                kx = max(kx, (uint64_t)__shfl_xor(kx, off, 64));
            }
        }
        if (lane == first) {
            add(v0, (unsigned)__popcll(mm));
            wit(v0, i);
            if (d < 8) minmax(v0, kn, kx);
        }
    } else if (match) {
        add(v, 1u);
        wit(v, i);
        if (d < 8) minmax(v, k, k);
    }
}

// The decision of one pass, by the 64 lanes of one wave: bin v holding rank
// s.rr (count(v), witness(v), kmin(v), kmax(v) read through the accessors),
// then the new state.  Returns the threshold's candidate index in *thr when
// the bin holds one candidate; sets *err for an inconsistency.  Exactly one
// lane updates s, *thr and *err, and returns true.
template <class Count, class Witness, class KMin, class KMax>
__device__ __forceinline__ bool narrow_decide(Narrow &s, int lane, const Cand &c, Count count,
                                              Witness witness, KMin kmin, KMax kmax,
                                              int64_t *thr, int *err) {
    unsigned hv[4], sum = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        hv[q] = count(4 * lane + q);
        sum += hv[q];
    }
    int64_t incl = sum;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int64_t o = __shfl_up(incl, off, 64);
        if (lane >= off) incl += o;
    }
    const int64_t rr = s.rr;
    const int d = s.d;
    int64_t base = incl - sum;
    int found = 0, vsel = 0;
    int64_t rnew = 0, cnt = 0;
    if (base <= rr && rr < incl) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            if (base <= rr && rr < base + (int64_t)hv[q]) {
                found = 1;
                vsel = 4 * lane + q;
                rnew = rr - base;
                cnt = hv[q];
            }
            base += hv[q];
        }
    }
    const uint64_t fm = __ballot(found);
    if (fm == 0) {
        if (lane != 0) return false;
        *err |= 16;  // rank outside the list: unreachable
        s.done = 1;
        return true;
    }
    if (lane != __ffsll((long long)fm) - 1) return false;
    const int sh = 56 - 8 * (d & 7);
    if (d < 8) {
        s.pk |= (uint64_t)vsel << sh;
        s.mk |= 0xffull << sh;
    } else {
        s.ph |= (uint64_t)vsel << sh;
        s.mh |= 0xffull << sh;
    }
    s.rr = rnew;
    if (cnt == 1) {
        const int64_t w = witness(vsel);
        if (w >= 0 && w < c.n) {
            *thr = w;
        } else {
            *err |= 16;
        }
        s.done = 1;
    } else if (d < 8) {
        const uint64_t lo = kmin(vsel), hi = kmax(vsel);
        if (lo == hi) {  // every key of the bucket is lo: on to the hash
            s.pk = lo;
            s.mk = ~0ull;
            s.d = 8;
        } else {
            const int j = __clzll((long long)(lo ^ hi)) >> 3;  // first byte where they differ
            s.pk = lo & top_bytes(j);
            s.mk = top_bytes(j);
            s.d = j;
        }
    } else if (d == 15) {
        *err |= 1;  // composites are unique: unreachable
        s.done = 1;
    } else {
        s.d = d + 1;
    }
    return true;
}

// The bin of one pass's histogram holding rank s.rr, by the 64 lanes of one
// wave: fixes digit s.d of the bucket to it and takes the rank within it.
// When the bin holds one candidate its index goes to *thr and s.done is set;
// *err records an inconsistency.
template <class Count, class Witness>
__device__ __forceinline__ void choose_bin(Narrow &s, int lane, const Cand &c, Count count,
                                           Witness witness, int64_t *thr, int *err) {
    unsigned hv[4], sum = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        hv[q] = count(4 * lane + q);
        sum += hv[q];
    }
    int64_t incl = sum;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int64_t o = __shfl_up(incl, off, 64);
        if (lane >= off) incl += o;
    }
    const int64_t rr = s.rr;
    int64_t base = incl - sum;
    int found = 0, vsel = 0;
    int64_t rnew = 0, cnt = 0;
    if (base <= rr && rr < incl) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            if (base <= rr && rr < base + (int64_t)hv[q]) {
                found = 1;
                vsel = 4 * lane + q;
                rnew = rr - base;
                cnt = hv[q];
            }
            base += hv[q];
        }
    }
    const uint64_t fm = __ballot(found);
    if (fm == 0) {
        if (lane == 0) {
            *err |= 16;  // rank outside the list: unreachable
            s.done = 1;
        }
        return;
    }
    const int src = __ffsll((long long)fm) - 1;
    if (lane == src) {
        const int d = s.d, sh = 56 - 8 * (d & 7);
        if (d < 8) {
            s.pk |= (uint64_t)vsel << sh;
            s.mk |= 0xffull << sh;
        } else {
            s.ph |= (uint64_t)vsel << sh;
            s.mh |= 0xffull << sh;
        }
        s.rr = rnew;
        if (cnt == 1) {
            const int64_t w = witness(vsel);
            if (w >= 0 && w < c.n) {
                *thr = w;
            } else {
                *err |= 16;
            }
            s.done = 1;
        }
    }
}

// Histogram contribution of one candidate without key ranges (all lanes of
// the wave call this together).
template <class AddCount, class SetWitness>
__device__ __forceinline__ void count_candidate(bool match, uint64_t k, uint64_t h, int d,
                                                int64_t i, AddCount add, SetWitness wit) {
    const uint32_t v = digit(k, h, d);
    const uint64_t mm = __ballot(match);
    if (mm == 0) return;
    const int first = __ffsll((long long)mm) - 1;
    const uint32_t v0 = __shfl(v, first, 64);
    if (__ballot(match && v == v0) == mm) {
        if ((int)(threadIdx.x & 63) == first) {
            add(v0, (unsigned)__popcll(mm));
            wit(v0, i);
        }
    } else if (match) {
        add(v, 1u);
        wit(v, i);
    }
}

// Block b finds the composite of rank r of list b (RESUME: continues the
// select from the state the multi-block passes left, when they did not
// finish).  With CACHED > 0 every thread keeps its (at most CACHED)
// candidates in registers for all the passes (lists of at most
// CACHED * kNarrowThreads entries); otherwise each pass reads the list again.
// Each pass histograms the current digit of the bucket's candidates; while
// the digit is a key byte, a second sweep over the bucket then takes the
// smallest and largest key of the chosen bin (one wave reduction per wave,
// not per candidate), and the select jumps past the bytes those share.
template <int CACHED, bool RESUME>
__global__ __launch_bounds__(kNarrowThreads) void narrow_kernel(Cand c0, Cand c1, int64_t r,
                                                                SelState *st) {
    const Cand c = blockIdx.x == 0 ? c0 : c1;
    const int b = blockIdx.x, tid = threadIdx.x, lane = tid & 63;
    if (RESUME && st->nar[b].done) return;  // the passes found it: same for every thread
    __shared__ unsigned hist[256];
    __shared__ int64_t witness[256];
    __shared__ unsigned long long s_lo, s_hi;
    __shared__ Narrow ns;
    __shared__ int64_t s_thr;
    __shared__ int s_err;
    if (tid == 0) {
        if (RESUME) {
            ns = st->nar[b];  // where the multi-block passes stopped
        } else {
            ns.pk = ns.ph = ns.mk = ns.mh = 0ull;
            ns.rr = r;
            ns.d = 0;
            ns.done = 0;
        }
        s_thr = -1;
        s_err = 0;
    }
    constexpr int NC = CACHED > 0 ? CACHED : 1;
    uint64_t ck[NC], ch[NC];
    if (CACHED > 0) {
#pragma unroll
        for (int u = 0; u < NC; ++u) {
            const int64_t i = u * kNarrowThreads + tid;
            ck[u] = i < c.n ? c.key[i] : 0ull;
            ch[u] = i < c.n ? c.hash[i] : 0ull;
        }
    }
    auto add = [&](int v, unsigned n) { atomicAdd(&hist[v], n); };
    auto wit = [&](int v, int64_t i) { witness[v] = i; };
    // f(key, hash, index) for every candidate of the list, all threads together
    auto each = [&](auto &&f) {
        if (CACHED > 0) {
#pragma unroll
            for (int u = 0; u < NC; ++u) f(ck[u], ch[u], u * kNarrowThreads + tid);
        } else {
            // four candidates per thread per iteration (loads in flight together)
            for (int64_t base = 0; base < c.n; base += 4 * kNarrowThreads) {
                uint64_t k[4], h[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int64_t i = base + u * kNarrowThreads + tid;
                    k[u] = i < c.n ? c.key[i] : 0ull;
                    h[u] = i < c.n ? c.hash[i] : 0ull;
                }
#pragma unroll
                for (int u = 0; u < 4; ++u) f(k[u], h[u], base + u * kNarrowThreads + tid);
            }
        }
    };
    for (int pass = 0; pass < 16; ++pass) {
        if (tid < 256) {
            hist[tid] = 0u;
            witness[tid] = -1;
        }
        __syncthreads();  // also publishes ns
        {
            const uint64_t pk = ns.pk, ph = ns.ph, mk = ns.mk, mh = ns.mh;
            const int d = ns.d;
            each([&](uint64_t k, uint64_t h, int64_t i) {
                const bool m = i < c.n && ((k ^ pk) & mk) == 0 && ((h ^ ph) & mh) == 0;
                count_candidate(m, k, h, d, i, add, wit);
            });
        }
        __syncthreads();
        if (tid < 64) {
            choose_bin(
                ns, lane, c, [&](int v) { return hist[v]; }, [&](int v) { return witness[v]; },
                &s_thr, &s_err);
            if (lane == 0) {
                s_lo = ~0ull;
                s_hi = 0ull;
            }
        }
        __syncthreads();
        if (ns.done) break;  // the same for every thread
        const int d = ns.d;
        if (d < 8) {
            // key range of the chosen bin (the bucket with digit d fixed)
            const uint64_t pk = ns.pk, ph = ns.ph, mk = ns.mk, mh = ns.mh;
            uint64_t lo = ~0ull, hi = 0ull;
            each([&](uint64_t k, uint64_t h, int64_t i) {
                if (i < c.n && ((k ^ pk) & mk) == 0 && ((h ^ ph) & mh) == 0) {
                    lo = min(lo, k);
                    hi = max(hi, k);
                }
            });
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) {
                lo = min(lo, (uint64_t)__shfl_xor(lo, off, 64));
                hi = max(hi, (uint64_t)__shfl_xor(hi, off, 64));
            }
            if (lane == 0 && lo <= hi) {
                atomicMin(&s_lo, (unsigned long long)lo);
                atomicMax(&s_hi, (unsigned long long)hi);
            }
            __syncthreads();
            if (tid == 0) {
                const uint64_t L = s_lo, H = s_hi;
                if (L > H) {
                    s_err |= 16;  // an empty bucket: unreachable
                    ns.done = 1;
                } else if (L == H) {  // every key of the bucket is L: on to the hash
                    ns.pk = L;
                    ns.mk = ~0ull;
                    ns.d = 8;
                } else {
                    const int j = __clzll((long long)(L ^ H)) >> 3;  // first differing byte
                    ns.pk = L & top_bytes(j);
                    ns.mk = top_bytes(j);
                    ns.d = j;
                }
            }
        } else if (tid == 0) {
            if (d == 15) {
                s_err |= 1;  // composites are unique: unreachable
                ns.done = 1;
            } else {
                ns.d = d + 1;
            }
        }
        __syncthreads();
        if (ns.done) break;
    }
    if (tid == 0) {
        if (s_err || !ns.done || s_thr < 0) {
            atomicOr(&st->error, s_err ? s_err : 1);
        } else {
            st->thr_key[b] = c.key[s_thr];
            st->thr_hash[b] = c.hash[s_thr];
        }
        st->count[b] = 0ull;
    }
}

// Multi-block narrowing for long lists: the same radix select, one launch per
// pass.  Every block adds its candidates' LDS histogram (counts, witnesses,
// key ranges) of the current digit into the list's; the last block to finish
// (a ticket counter) takes the decision and clears the histogram for the
// next launch.  Launches after the threshold is known return at once.
__global__ void narrow_init_kernel(SelState *st, int64_t r) {
    const int b = blockIdx.x, t = threadIdx.x;
    if (t < 256) {
        st->hist[b][t] = 0u;
        st->wit[b][t] = -1;
        st->kmin[b][t] = ~0ull;
        st->kmax[b][t] = 0ull;
    }
    if (t == 0) {
        Narrow &n = st->nar[b];
        n.pk = n.ph = n.mk = n.mh = 0ull;
        n.rr = r;
        n.d = 0;
        n.done = 0;
        st->ticket[b] = 0u;
        st->count[b] = 0ull;
    }
}

__global__ __launch_bounds__(kPassThreads) void narrow_pass_kernel(Cand c0, Cand c1,
                                                                   SelState *st) {
    const int b = blockIdx.y, tid = threadIdx.x, lane = tid & 63;
    if (st->nar[b].done) return;  // the same for every thread of the launch
    const Cand c = b == 0 ? c0 : c1;
    const Narrow ns = st->nar[b];
    __shared__ unsigned hist[256];
    __shared__ int64_t witness[256];
    __shared__ unsigned long long kmin[256], kmax[256];
    __shared__ int last;
    hist[tid] = 0u;
    witness[tid] = -1;
    kmin[tid] = ~0ull;
    kmax[tid] = 0ull;
    __syncthreads();
    auto add = [&](int v, unsigned n) { atomicAdd(&hist[v], n); };
    auto wit = [&](int v, int64_t i) { witness[v] = i; };
    auto minmax = [&](int v, uint64_t lo, uint64_t hi) {
        atomicMin(&kmin[v], (unsigned long long)lo);
        atomicMax(&kmax[v], (unsigned long long)hi);
    };
    const int64_t stride = (int64_t)gridDim.x * kPassThreads;
    for (int64_t base = (int64_t)blockIdx.x * kPassThreads; base < c.n; base += stride) {
        const int64_t i = base + tid;
        const uint64_t k = i < c.n ? c.key[i] : 0ull, h = i < c.n ? c.hash[i] : 0ull;
        const bool m = i < c.n && ((k ^ ns.pk) & ns.mk) == 0 && ((h ^ ns.ph) & ns.mh) == 0;
        bin_candidate(m, k, h, ns.d, i, lane, add, wit, minmax);
    }
    __syncthreads();
    if (hist[tid]) {
        atomicAdd(&st->hist[b][tid], hist[tid]);
        // read only when the bin holds one candidate
        atomicExch((unsigned long long *)&st->wit[b][tid], (unsigned long long)witness[tid]);
        if (ns.d < 8) {
            atomicMin((unsigned long long *)&st->kmin[b][tid], kmin[tid]);
            atomicMax((unsigned long long *)&st->kmax[b][tid], kmax[tid]);
        }
    }
    __threadfence();
    __syncthreads();
    if (tid == 0) last = atomicAdd(&st->ticket[b], 1u) == gridDim.x - 1;
    __syncthreads();
    if (!last) return;
    __threadfence();
    if (tid < 64) {
        // the list's histogram, read at the device scope where the other
        // blocks' atomics landed
        Narrow n = ns;
        int64_t thr = -1;
        int err = 0;
        const bool decided = narrow_decide(
            n, lane, c, [&](int v) { return atomicAdd(&st->hist[b][v], 0u); },
            [&](int v) {
                return (int64_t)atomicAdd((unsigned long long *)&st->wit[b][v], 0ull);
            },
            [&](int v) { return (uint64_t)atomicAdd((unsigned long long *)&st->kmin[b][v], 0ull); },
            [&](int v) { return (uint64_t)atomicAdd((unsigned long long *)&st->kmax[b][v], 0ull); },
            &thr, &err);
        // the deciding lane publishes the new state
        if (decided) {
            st->nar[b] = n;
            if (err) atomicOr(&st->error, err);
            if (thr >= 0) {
                st->thr_key[b] = c.key[thr];
                st->thr_hash[b] = c.hash[thr];
            }
        }
    }
    __syncthreads();  // the decision has read the histogram
    // clear the histogram and the ticket for the next launch
    atomicExch(&st->hist[b][tid], 0u);
    atomicExch((unsigned long long *)&st->kmin[b][tid], ~0ull);
    atomicExch((unsigned long long *)&st->kmax[b][tid], 0ull);
    if (tid == 0) atomicExch(&st->ticket[b], 0u);
}

// Candidates of list blockIdx.y with composite in (lo, thr] (lo only when
// has_lo) into the dense chunk lists; slots claimed with one atomic per block.
constexpr int kCompactThreads = 1024;
__global__ __launch_bounds__(kCompactThreads) void compact_kernel(Cand c0, Cand c1, int has_lo,
                                                                  SelState *st, uint64_t *ck,
                                                                  uint64_t *chh, int32_t *ci,
                                                                  int64_t cap) {
    const int b = blockIdx.y;
    const Cand c = b == 0 ? c0 : c1;
    const int64_t i = (int64_t)blockIdx.x * kCompactThreads + threadIdx.x;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    __shared__ unsigned wave_n[kCompactThreads / 64];
    __shared__ unsigned long long block_base;
    bool take = false;
    uint64_t k = 0, h = 0;
    if (i < c.n) {
        k = c.key[i];
        h = c.hash[i];
        take = !less128(st->thr_key[b], st->thr_hash[b], k, h) &&
               (!has_lo || less128(st->lo_key[b], st->lo_hash[b], k, h));
    }
    const uint64_t m = __ballot(take);
    if (lane == 0) wave_n[w] = (unsigned)__popcll(m);
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long tot = 0;
        for (int q = 0; q < kCompactThreads / 64; ++q) tot += wave_n[q];
        block_base = tot ? atomicAdd(&st->count[b], tot) : 0ull;
    }
    __syncthreads();
    if (!take) return;
    unsigned long long slot = block_base + __popcll(m & ((1ull << lane) - 1ull));
    for (int q = 0; q < w; ++q) slot += wave_n[q];
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

// Multi-block pass launches before the one-workgroup finish
// (LBM_NARROW_PASSES overrides it, 0..16).
static int pass_launches() {
    static const int v = [] {
        const char *e = std::getenv("LBM_NARROW_PASSES");
        return e ? std::min(16, std::max(0, std::atoi(e))) : kPassLaunches;
    }();
    return v;
}

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
        if (nmax <= kNarrowCached * kNarrowThreads) {
            hipLaunchKernelGGL((narrow_kernel<kNarrowCached, false>), dim3(2),
                               dim3(kNarrowThreads), 0, s, c0, c1, hi - 1, st);
        } else {
            // long lists: a few multi-block launches, one per byte, then one
            // workgroup per list finishes the select if they did not
            const unsigned blocks = (unsigned)std::min<int64_t>(
                kMaxPassBlocks, (nmax + 4 * kPassThreads - 1) / (4 * kPassThreads));
            hipLaunchKernelGGL(narrow_init_kernel, dim3(2), dim3(256), 0, s, st, hi - 1);
            for (int pass = 0; pass < pass_launches(); ++pass)
                hipLaunchKernelGGL(narrow_pass_kernel, dim3(blocks, 2), dim3(kPassThreads), 0, s,
                                   c0, c1, st);
            hipLaunchKernelGGL((narrow_kernel<0, true>), dim3(2), dim3(kNarrowThreads), 0, s, c0,
                               c1, hi - 1, st);
        }
        hipLaunchKernelGGL(zero_u32_kernel, dim3((unsigned)std::min<int64_t>(1024, (2 * m + 255) / 256)),
                           dim3(256), 0, s, rank, 2 * L.cap);
        hipLaunchKernelGGL(compact_kernel,
                           dim3((unsigned)((nmax + kCompactThreads - 1) / kCompactThreads), 2),
                           dim3(kCompactThreads), 0, s, c0, c1, lo > 0 ? 1 : 0, st, ck, chh, ci,
                           L.cap);
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
