// Candidate keys and flips of the exchange step (Sec. 2.2, Eqs. 5-6; Sec. 2.3
// steps 3-4), shared by the storage forms.
//
// The keys need the density and velocity of each interface cell and of the
// non-solid neighbours of each solid interface cell.  They are taken either
// from a caller-supplied field (logical layout, FIELD = true) or straight
// from the stored state through the storage form's moments policy M, which
// is the one its macroscopic export uses, so both give the same bits.  Only
// interface cells and their neighbours are read; no whole-lattice field is
// formed.
//
// M provides:  using T;  static void at(const T *f, size_t plane, size_t n,
//              double &rho, double &ux, double &uy)   (n: pitched index).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lbm_internal.h"

namespace lbm {
namespace keys {

__device__ __forceinline__ uint64_t splitmix64(uint64_t state) {
    // SplitMix64 output function (Steele, Lea & Flood 2014) on state + gamma
    uint64_t z = state + 0x9e3779b97f4a7c15ull;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

// Order-preserving integer image of a key >= 0 (-0 folded onto +0).
__device__ __forceinline__ uint64_t key_bits(double k) {
    return k == 0.0 ? 0ull : (uint64_t)__double_as_longlong(k);
}

// rho, ux, uy of cell (x, y): from the field or from the state.
template <class M, bool FIELD>
__device__ __forceinline__ void cell_field(const KeysArgs &a, int x, int y, double &rho,
                                           double &ux, double &uy) {
    if (FIELD) {
        const size_t l = (size_t)y * a.nx + x;
        rho = a.rho[l];
        ux = a.ux[l];
        uy = a.uy[l];
    } else {
        M::at(static_cast<const typename M::T *>(a.f), a.plane, (size_t)y * a.pitch + x, rho,
              ux, uy);
    }
}

// Key of cell (x, y) if it is an interface cell inside the band: 1 for a
// fluid candidate, 2 for a solid one, 0 otherwise; *bad when a key is NaN or
// negative.
template <class M, bool FIELD>
__device__ __forceinline__ int cell_key(const KeysArgs &a, int x, int y, double &key, bool &bad) {
#pragma clang fp contract(off)
    const int nx = a.nx;
    const bool in_band = x >= a.band_x && x <= a.nx - 1 - a.band_x && y >= a.band_y &&
                         y <= a.ny - 1 - a.band_y;
    if (!in_band) return 0;
    const size_t l = (size_t)y * nx + x;
    const uint8_t t = a.types[l];
    const int ddx[4] = {1, 0, -1, 0};
    const int ddy[4] = {0, 1, 0, -1};
    bool touch = false, nan = false;
    key = 0.0;
    if (t == kFluid) {
#pragma unroll
        for (int d = 0; d < 4; ++d)
            touch |= a.types[l + ddx[d] + (ptrdiff_t)ddy[d] * nx] == kSolid;
        if (touch) {
            double rho, ux, uy;
            cell_field<M, FIELD>(a, x, y, rho, ux, uy);
            const double t1 = ux * ux;
            const double t2 = uy * uy;
            const double t3 = t1 + t2;
            key = a.criterion == kCritPaper ? rho * t3 : t3;
        }
    } else if (t == kSolid) {
#pragma unroll
        for (int d = 0; d < 4; ++d) {
            const size_t m = l + ddx[d] + (ptrdiff_t)ddy[d] * nx;
            if (a.types[m] == kSolid) continue;
            touch = true;
            double rho, ux, uy;
            cell_field<M, FIELD>(a, x + ddx[d], y + ddy[d], rho, ux, uy);
            if (a.criterion == kCritPaper) {
                const double tang = ddx[d] != 0 ? fabs(uy) : fabs(ux);
                key = key + tang;
            } else {
                const double t1 = ux * ux;
                const double t2 = uy * uy;
                const double s = t1 + t2;
                if (!(s >= 0.0)) nan = true;
                if (s > key) key = s;
            }
        }
    }
    if (!touch) return 0;
    if (nan || !(key >= 0.0)) {
        bad = true;
        return 0;
    }
    return t == kFluid ? 1 : (t == kSolid ? 2 : 0);
}

// Candidate keys of the interface cells inside the band.  Fluid candidates
// sort ascending on (key, hash, idx); solid candidates descending on key,
// which is stored complemented so that both lists sort ascending.  A block
// of 64 x kRows threads covers 64 x (kRows kIter) cells (thread (lane, w)
// takes rows w, w + kRows, ...), and claims its candidates' list slots with
// one atomic per list: the list order is any order (the selection sorts).
// One row per thread: eight (one eighth of the atomics) measured 1.4-3x
// slower, the gathers of the interface cells' moments wanting the threads.
constexpr int kRows = 16, kIter = 1;
template <class M, bool FIELD>
__global__ __launch_bounds__(64 * kRows) void keys_kernel(KeysArgs a) {
    const int x = blockIdx.x * 64 + threadIdx.x;
    const int lane = threadIdx.x, w = threadIdx.y;
    const int y0 = blockIdx.y * kRows * kIter + w;
    double key[kIter];
    int kind[kIter];
    bool bad = false;
    unsigned nf = 0, ns = 0;  // the wave's candidates over its rows
#pragma unroll
    for (int it = 0; it < kIter; ++it) {
        kind[it] = cell_key<M, FIELD>(a, x, y0 + it * kRows, key[it], bad);
        nf += (unsigned)__popcll(__ballot(kind[it] == 1));
        ns += (unsigned)__popcll(__ballot(kind[it] == 2));
    }
    if (bad) atomicOr(a.error, 1);
    __shared__ unsigned wave_n[2][kRows];
    __shared__ unsigned long long block_base[2];
    if (lane == 0) {
        wave_n[0][w] = nf;
        wave_n[1][w] = ns;
    }
    __syncthreads();
    if (w == 0 && lane < 2) {
        unsigned long long tot = 0;
        for (int k = 0; k < kRows; ++k) tot += wave_n[lane][k];
        block_base[lane] = tot ? atomicAdd(lane == 0 ? a.count_f : a.count_s, tot) : 0ull;
    }
    __syncthreads();
    unsigned long long bf = block_base[0], bs = block_base[1];
    for (int k = 0; k < w; ++k) {
        bf += wave_n[0][k];
        bs += wave_n[1][k];
    }
    // slots in (row, lane) order within the wave
    const uint64_t below = (1ull << lane) - 1ull;
#pragma unroll
    for (int it = 0; it < kIter; ++it) {
        const uint64_t mf = __ballot(kind[it] == 1), ms = __ballot(kind[it] == 2);
        if (kind[it] != 0) {
            const size_t l = (size_t)(y0 + it * kRows) * a.nx + x;
            const uint64_t kb = key_bits(key[it]);
            const uint64_t h = splitmix64(a.seed + (uint64_t)l);
            if (kind[it] == 1) {
                const unsigned long long s = bf + (unsigned long long)__popcll(mf & below);
                if (s < (unsigned long long)a.cap) {
                    a.kf[s] = kb;
                    a.hf[s] = h;
                    a.if_[s] = (int32_t)l;
                }
            } else {
                const unsigned long long s = bs + (unsigned long long)__popcll(ms & below);
                if (s < (unsigned long long)a.cap) {
                    a.ks[s] = ~kb;
                    a.hs[s] = h;
                    a.is[s] = (int32_t)l;
                }
            }
        }
        bf += (unsigned long long)__popcll(mf);
        bs += (unsigned long long)__popcll(ms);
    }
}

// Flip the selected cells of the logical type map and record the density of
// each removed cell, in selection order (from the field, or from the state
// before the re-initialisation touches it).
template <class M, bool FIELD>
__global__ void flip_kernel(FlipArgs a) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= a.k_eff) return;
    const int32_t r = a.removed[k];
    if (FIELD) {
        a.removed_rho[k] = a.rho[r];
    } else {
        double rho, ux, uy;
        M::at(static_cast<const typename M::T *>(a.f), a.plane,
              (size_t)(r / a.nx) * a.pitch + (size_t)(r % a.nx), rho, ux, uy);
        a.removed_rho[k] = rho;
    }
    a.types[r] = kSolid;
    a.types[a.added[k]] = kFluid;
}

template <class M>
hipError_t launch_keys(const KeysArgs &a, hipStream_t s) {
    const dim3 grid((unsigned)((a.nx + 63) / 64),
                    (unsigned)((a.ny + kRows * kIter - 1) / (kRows * kIter)));
    if (a.rho)
        hipLaunchKernelGGL((keys_kernel<M, true>), grid, dim3(64, kRows), 0, s, a);
    else
        hipLaunchKernelGGL((keys_kernel<M, false>), grid, dim3(64, kRows), 0, s, a);
    return hipGetLastError();
}

template <class M>
hipError_t launch_flip(const FlipArgs &a, hipStream_t s) {
    if (a.k_eff <= 0) return hipSuccess;
    const dim3 grid((unsigned)((a.k_eff + 255) / 256));
    if (a.rho)
        hipLaunchKernelGGL((flip_kernel<M, true>), grid, dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL((flip_kernel<M, false>), grid, dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace keys
}  // namespace lbm
