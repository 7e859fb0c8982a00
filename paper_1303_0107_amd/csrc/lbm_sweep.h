// The D2Q9 time-step kernels, generic in the per-cell arithmetic.
//
// A `Cell` policy supplies the storage type T, the arithmetic type CT, the
// conversions Cell::load (T -> CT) and Cell::store (CT -> T), and the update
// of one cell:
//     Cell::update(CT (&f)[9], type, uin, args, mass, ux, uy)
// turns the nine pulled populations (after streaming, before the boundary
// closure) into the post-collision populations, and reports the cell's
// density and velocity.  Two kernels share it, so both produce the same bits:
//
//   step_kernel  one time step, one lane per cell, read the source buffer and
//                write the other (ping-pong).
//   tb_kernel    temporal blocking: a workgroup loads a 64 x RH region (its
//                64-2H x RH-2H tile plus a halo of H cells) into LDS,
//                advances it up to H steps in place, and writes back its tile.
//                After s steps only cells at least s cells inside the region
//                are valid; a tile cell is at least H inside, so it is valid
//                after every step count up to H.  Launch cost and DRAM
//                latency are paid once per H steps, and the populations cross
//                HBM once per launch instead of once per step.
//
// Pull streaming (Eq. 1): population i of cell x comes from cell x - c_i,
// or, when bit i-1 of the cell word flags that link as cut by a wall, from
// population opp(i) of x itself (halfway bounce-back).  Cell words:
// bits 0..7 wall flags of populations 1..8, bits 8..9 the cell type.
//
// This header is included by one translation unit per precision, after that
// unit has set its floating-point contraction mode.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lbm_internal.h"

namespace lbm {
namespace sweep {

__device__ constexpr int kCx[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
__device__ constexpr int kCy[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
__device__ constexpr int kOpp[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};

// Sum of NV doubles over a block of NT threads into thread 0, in a fixed
// order (wave butterflies, then waves in index order).
template <int NV, int NT>
__device__ __forceinline__ void block_sum(double (&v)[NV]) {
    __shared__ double red[NT / 64][NV];
    const int tid = threadIdx.y * blockDim.x + threadIdx.x;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
#pragma unroll
        for (int k = 0; k < NV; ++k) v[k] += __shfl_xor(v[k], off, 64);
    if ((tid & 63) == 0)
#pragma unroll
        for (int k = 0; k < NV; ++k) red[tid >> 6][k] = v[k];
    __syncthreads();
    if (tid == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) {
            double s = red[0][k];
            for (int w = 1; w < NT / 64; ++w) s += red[w][k];
            v[k] = s;
        }
    }
}

// Residual terms of one cell (|u - u_prev|^2, |u|^2, rho, non-finite count)
// added to `part`; u_prev is replaced by u.
template <typename T>
__device__ __forceinline__ void check_terms(const SweepArgs<T> &a, size_t n,
                                            double mass, double ux, double uy,
                                            double (&part)[4]) {
    const double px = a.uprev[n], py = a.uprev[a.plane + n];
    const double dx = ux - px, dy = uy - py;
    part[0] += dx * dx + dy * dy;
    part[1] += ux * ux + uy * uy;
    part[2] += mass;
    part[3] += (isfinite(mass) && isfinite(ux) && isfinite(uy)) ? 0.0 : 1.0;
    a.uprev[n] = ux;
    a.uprev[a.plane + n] = uy;
}

template <class Cell, bool CHECK>
__global__ __launch_bounds__(256) void step_kernel(SweepArgs<typename Cell::T> a) {
    using T = typename Cell::T;
    using CT = typename Cell::CT;
    const int x = blockIdx.x * 64 + threadIdx.x;
    const int y = blockIdx.y * 4 + threadIdx.y;
    const bool in = x < a.nx && y < a.ny;
    const size_t n = (size_t)(in ? y : 0) * a.pitch + (in ? x : 0);
    const uint32_t cw = in ? a.cell[n] : 0u;
    const uint32_t type = cw >> 8;
    double part[4] = {0.0, 0.0, 0.0, 0.0};
    if (in && type != kSolid) {
        const size_t P = a.plane;
        CT f[9];
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            const bool wall = i > 0 && ((cw >> (i - 1)) & 1u);
            const size_t src = wall ? (size_t)kOpp[i] * P + n
                                    : (size_t)i * P + n - kCx[i] - (ptrdiff_t)kCy[i] * a.pitch;
            f[i] = Cell::load(a.fin[src]);
        }
        double mass, ux, uy;
        Cell::update(f, type, type == kInlet ? (CT)a.uin[y] : CT(0), a, mass, ux, uy);
#pragma unroll
        for (int i = 0; i < 9; ++i) a.fout[(size_t)i * P + n] = Cell::store(f[i]);
        if (CHECK) check_terms(a, n, mass, ux, uy, part);
    }
    if (CHECK) {
        block_sum<4, 256>(part);
        if (threadIdx.x == 0 && threadIdx.y == 0) {
            const size_t b = (size_t)blockIdx.y * gridDim.x + blockIdx.x;
#pragma unroll
            for (int k = 0; k < 4; ++k) a.partials[b * 4 + k] = part[k];
        }
    }
}

// Temporal blocking.  Tile t = tiles[blockIdx.x] packs (tile row << 16 | tile
// column); the tile's cells are [tx*IW, tx*IW+IW) x [ty*IH, ty*IH+IH).
// Lane l of wave w owns region cells (l, w + c*NW), c = 0..CPT-1.
// PP (ping-pong): two LDS copies of the region, each step reads one and
// writes the other (one barrier per step, nothing held in registers across
// the barrier).  Otherwise one copy updated in place: every thread keeps its
// cells' new populations in registers until all reads of the step are done.
template <class Cell, int RH, int H, int NT, bool PP, bool CHECK>
__global__ __launch_bounds__(NT) void tb_kernel(SweepArgs<typename Cell::T> a,
                                                const int32_t *__restrict__ tiles,
                                                int steps) {
    using T = typename Cell::T;
    using CT = typename Cell::CT;
    constexpr int RW = 64, IW = RW - 2 * H, IH = RH - 2 * H;
    constexpr int NW = NT / 64, CPT = RH / NW, PL = RW * RH;
    static_assert(RH % NW == 0, "region rows must split evenly over waves");
    extern __shared__ __align__(16) unsigned char lds_raw[];
    T *L = reinterpret_cast<T *>(lds_raw);

    const int t = tiles[blockIdx.x];
    const int ox = (t & 0xffff) * IW - H, oy = (t >> 16) * IH - H;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int gx = ox + lane;
    const bool col_in = gx >= 0 && gx < a.nx;

    uint32_t cw[CPT];
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
        const int ry = wave + c * NW, gy = oy + ry;
        const bool in = col_in && gy >= 0 && gy < a.ny;
        const size_t n = in ? (size_t)gy * a.pitch + gx : 0;
        cw[c] = in ? a.cell[n] : 0u;
        const bool live = in && (cw[c] >> 8) != kSolid;
#pragma unroll
        for (int i = 0; i < 9; ++i)
            L[i * PL + ry * RW + lane] = live ? a.fin[(size_t)i * a.plane + n] : Cell::store(CT(0));
    }
    __syncthreads();

    double part[4] = {0.0, 0.0, 0.0, 0.0};
    int src_buf = 0;
    for (int s = 1; s <= steps; ++s) {
        const bool last = s == steps;
        const T *Ls = L + (PP ? src_buf * 9 * PL : 0);
        T *Ld = L + (PP ? (1 - src_buf) * 9 * PL : 0);
        T out[PP ? 1 : CPT][9];
        bool upd[CPT];
#pragma unroll
        for (int c = 0; c < CPT; ++c) {
            const int ry = wave + c * NW;
            const uint32_t type = cw[c] >> 8;
            bool v = type != kSolid && lane >= s && lane < RW - s && ry >= s && ry < RH - s;
            if (last) v = v && lane >= H && lane < H + IW && ry >= H && ry < H + IH;
            upd[c] = v;
            if (v) {
                CT f[9];
#pragma unroll
                for (int i = 0; i < 9; ++i) {
                    const bool wall = i > 0 && ((cw[c] >> (i - 1)) & 1u);
                    const int src = wall ? kOpp[i] * PL + ry * RW + lane
                                         : i * PL + (ry - kCy[i]) * RW + lane - kCx[i];
                    f[i] = Cell::load(Ls[src]);
                }
                double mass, ux, uy;
                const int gy = oy + ry;
                Cell::update(f, type, type == kInlet ? (CT)a.uin[gy] : CT(0), a, mass, ux, uy);
                if (last) {
                    const size_t n = (size_t)gy * a.pitch + gx;
#pragma unroll
                    for (int i = 0; i < 9; ++i) a.fout[(size_t)i * a.plane + n] = Cell::store(f[i]);
                    if (CHECK) check_terms(a, n, mass, ux, uy, part);
                } else if (PP) {
#pragma unroll
                    for (int i = 0; i < 9; ++i) Ld[i * PL + ry * RW + lane] = Cell::store(f[i]);
                } else {
#pragma unroll
                    for (int i = 0; i < 9; ++i) out[PP ? 0 : c][i] = Cell::store(f[i]);
                }
            }
        }
        if (last) break;
        if (!PP) {
            __syncthreads();
#pragma unroll
            for (int c = 0; c < CPT; ++c)
                if (upd[c]) {
                    const int ry = wave + c * NW;
#pragma unroll
                    for (int i = 0; i < 9; ++i) L[i * PL + ry * RW + lane] = out[PP ? 0 : c][i];
                }
        }
        __syncthreads();
        src_buf = 1 - src_buf;
    }
    if (CHECK) {
        block_sum<4, NT>(part);
        if (threadIdx.x == 0) {
#pragma unroll
            for (int k = 0; k < 4; ++k) a.partials[(size_t)blockIdx.x * 4 + k] = part[k];
        }
    }
}

// Host-side launch helpers shared by the per-precision units.
template <class Cell>
hipError_t launch_step(const SweepArgs<typename Cell::T> &a, bool check, hipStream_t s) {
    const dim3 g((unsigned)((a.nx + 63) / 64), (unsigned)((a.ny + 3) / 4)), b(64, 4);
    if (check)
        hipLaunchKernelGGL((step_kernel<Cell, true>), g, b, 0, s, a);
    else
        hipLaunchKernelGGL((step_kernel<Cell, false>), g, b, 0, s, a);
    return hipGetLastError();
}

template <class Cell, int RH, int H, int NT, bool PP>
hipError_t launch_tb(const SweepArgs<typename Cell::T> &a, const int32_t *tiles, int n_tiles,
                     int steps, bool check, hipStream_t s) {
    if (n_tiles <= 0 || steps <= 0) return hipSuccess;
    if (steps > H) return hipErrorInvalidValue;
    const size_t lds = (size_t)(PP ? 2 : 1) * 9 * 64 * RH * sizeof(typename Cell::T);
    auto k_plain = tb_kernel<Cell, RH, H, NT, PP, false>;
    auto k_check = tb_kernel<Cell, RH, H, NT, PP, true>;
    static bool configured = false;
    if (!configured) {
        hipError_t e = hipFuncSetAttribute((const void *)k_plain,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        e = hipFuncSetAttribute((const void *)k_check,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        configured = true;
    }
    if (check)
        hipLaunchKernelGGL(k_check, dim3((unsigned)n_tiles), dim3(NT), lds, s, a, tiles, steps);
    else
        hipLaunchKernelGGL(k_plain, dim3((unsigned)n_tiles), dim3(NT), lds, s, a, tiles, steps);
    return hipGetLastError();
}

}  // namespace sweep
}  // namespace lbm
