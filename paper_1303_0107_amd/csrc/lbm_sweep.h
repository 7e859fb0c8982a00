// The D2Q9 time-step kernels, generic in the per-cell arithmetic.
//
// A `Cell` policy supplies the storage type T, the arithmetic type CT, the
// conversions Cell::load (T -> CT) and Cell::store (CT -> T), and the update
// of one cell:
//     Cell::update(CT (&f)[9], type, bx, by, args, mass, ux, uy)
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

#include <type_traits>

#include "lbm_internal.h"

namespace lbm {
namespace sweep {

__device__ constexpr int kCx[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
__device__ constexpr int kCy[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
__device__ constexpr int kOpp[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
// mirror image of c_i under y -> -y
__device__ constexpr int kMirY[9] = {0, 1, 4, 3, 2, 8, 7, 6, 5};

// Pull source of population i for a cell flagged kWordGeneral (top row under
// a symmetry plane), as an offset (plane, row, column) into an array of row
// stride `stride`: a source beyond the symmetry line above row ny-1 is the
// mirror population (c_y reversed) of the cell in row ny-1 (gy is the cell's
// lattice row, ry its array row).
__device__ __forceinline__ size_t general_src(uint32_t cw, int i, int col, int ry, int gy,
                                              int ny, int flags, size_t plane, int stride) {
    const bool wall = i > 0 && ((cw >> (i - 1)) & 1u);
    if (wall) return (size_t)kOpp[i] * plane + (size_t)ry * stride + col;
    int rs = ry - kCy[i], pop = i;
    if ((flags & kFlagSymmetryTop) && gy - kCy[i] == ny) {
        rs = ry;
        pop = kMirY[i];
    }
    return (size_t)pop * plane + (size_t)rs * stride + (col - kCx[i]);
}

// LDS stores of one region cell in a step: plane i of copy b sits at
// (2i + b) * PL elements, reached from one of three LDS addresses (planes 0-3,
// 4-7, 8), so that every store's remaining offset fits the 16-bit immediate
// of an LDS instruction.  The addresses are made opaque once per launch so
// that they stay in registers instead of being recomputed at every step.
template <typename T, int PL>
struct StoreBases {
    // the stored bits (the 16-bit formats are classes without an assignment
    // in the LDS address space)
    using Bits = typename std::conditional<
        sizeof(T) == 8, uint64_t,
        typename std::conditional<sizeof(T) == 4, uint32_t, uint16_t>::type>::type;
    using LdsBits = __attribute__((address_space(3))) Bits;
    LdsBits *b[3];
    __device__ __forceinline__ void set(T *L, int pos) {
        LdsBits *p = (LdsBits *)reinterpret_cast<Bits *>(L + pos);
        b[0] = p;
        b[1] = p + 8 * PL;
        b[2] = p + 16 * PL;
#pragma unroll
        for (int k = 0; k < 3; ++k) asm volatile("" : "+v"(b[k]));
    }
    // Population i into copy C.
    template <int C>
    __device__ __forceinline__ void put(int i, T v) const {
        Bits w;
        __builtin_memcpy(&w, &v, sizeof(T));
        if (i < 4)
            b[0][(2 * i + C) * PL] = w;
        else if (i < 8)
            b[1][(2 * (i - 4) + C) * PL] = w;
        else
            b[2][C * PL] = w;
    }
};

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

// Stop decision of a check interval from its four sums (residual numerator
// and denominator, mass, non-finite count): 2 when the run became unstable
// (a non-finite sum, or a non-finite cell flagged), 1 when it converged (tol
// > 0 and sqrt(num)/sqrt(den) < tol), else 0.
__device__ __forceinline__ int interval_stop(const double (&v)[4], double tol) {
    const double num = v[0], den = v[1], bad = v[3];
    if (bad != 0.0 || !isfinite(num) || !isfinite(den)) return 2;
    if (tol > 0.0) {
        const double r = den == 0.0 ? (num == 0.0 ? 0.0 : INFINITY) : sqrt(num) / sqrt(den);
        if (r < tol) return 1;
    }
    return 0;
}

// Records interval j of a queued run (one thread): its sums, the count of
// intervals carried out, and the stop flag, with its lane copies in lanes0
// and, if given, lanes1.
__device__ __forceinline__ void record_interval(RunControl *ctl, int j, const double (&v)[4],
                                                int stop, int *lanes0, int *lanes1) {
#pragma unroll
    for (int k = 0; k < 4; ++k) ctl->sums[j][k] = v[k];
    ctl->done = j + 1;
    if (stop) {
        ctl->stop = stop;
        for (int l = 0; l < 64; ++l) {
            lanes0[l] = stop;
            if (lanes1) lanes1[l] = stop;
        }
    }
}

// Start of a blocked launch that may belong to a queued run (HALT).  The
// run's stop flag and, on the first launch of an interval that decides the
// interval before it (PREV, SweepArgs::prev), that interval's partials are
// read at the start, beside the region.  The workgroup leaves before its
// first barrier when the run had already ended, and right after it when the
// previous interval ends the run; no global store precedes either exit.
// The previous interval is summed in finalize_check_kernel's order (threads
// 0-255 add partials t and t + 256, the waves add their lanes, then the four
// wave sums are added in wave order), so every workgroup reaches the sums,
// bit for bit, that a finalize launch would record; workgroup 0 records
// them and writes the stop flag (the decision, or the flag it read) to the
// lane copies the interval's later launches read (SweepArgs::stop_out).
template <int NT, bool HALT, bool PREV>
struct RunGate {
    static_assert(!PREV || NT >= 256, "the previous interval's sum order takes 256 threads");
    int halt = 0;
    double p[2][4];

    template <typename T>
    __device__ __forceinline__ void read(const SweepArgs<T> &a) {
        if (!HALT) return;
        halt = a.stop[threadIdx.x & 63];
        if (!PREV) return;
        const int t = threadIdx.x;
#pragma unroll
        for (int r = 0; r < 2; ++r) {
            const bool in = t < 256 && t + 256 * r < a.prev_count;
#pragma unroll
            for (int k = 0; k < 4; ++k) p[r][k] = in ? a.prev[(size_t)(t + 256 * r) * 4 + k] : 0.0;
        }
    }

    static __device__ __forceinline__ double (*wave_sums())[4] {
        __shared__ double s[4][4];
        return s;
    }

    // Before the first barrier: true when the run had already ended (the
    // flag is the same for every lane).
    template <typename T>
    __device__ __forceinline__ bool ended(const SweepArgs<T> &a) {
        if (!HALT) return false;
        const int t = threadIdx.x;
        if (__builtin_amdgcn_readfirstlane(halt)) {
            if (PREV && blockIdx.x == 0 && t < 64) a.stop_out[t] = halt;  // passed on
            return true;
        }
        if (PREV && t < 256) {
            double v[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int r = 0; r < 2; ++r)
                if (t + 256 * r < a.prev_count)
#pragma unroll
                    for (int k = 0; k < 4; ++k) v[k] += p[r][k];
#pragma unroll
            for (int off = 32; off > 0; off >>= 1)
#pragma unroll
                for (int k = 0; k < 4; ++k) v[k] += __shfl_xor(v[k], off, 64);
            if ((t & 63) == 0)
#pragma unroll
                for (int k = 0; k < 4; ++k) wave_sums()[t >> 6][k] = v[k];
        }
        return false;
    }

    // After the first barrier: true when the previous interval ends the run.
    // Wave 0 alone forms the totals and the decision and hands the decision
    // to the other waves through LDS (one more barrier, in this launch only).
    template <typename T>
    __device__ __forceinline__ bool ends_now(const SweepArgs<T> &a) {
        if (!HALT || !PREV) return false;
        __shared__ int s_stop;
        if (threadIdx.x < 64) {
            double v[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                double s = wave_sums()[0][k];
                for (int w = 1; w < 4; ++w) s += wave_sums()[w][k];
                v[k] = s;
            }
            const int stop = interval_stop(v, a.tol);
            if (threadIdx.x == 0) {
                s_stop = stop;
                if (blockIdx.x == 0) record_interval(a.ctl, a.prev_j, v, stop, a.stop_out, nullptr);
            }
        }
        __syncthreads();
        return s_stop != 0;
    }
};

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

// One time step of the 64 x 4 cells of block (bx, by).  BC: the lattice has
// boundary-variant cells (flags != 0); without them those paths compile out.
template <class Cell, bool CHECK, bool BC>
__device__ __forceinline__ void step_body(const SweepArgs<typename Cell::T> &a, const int bx,
                                          const int by, double *part_out) {
    using CT = typename Cell::CT;
    const int x = bx * 64 + threadIdx.x;
    const int y = by * 4 + threadIdx.y;
    const bool in = x < a.nx && y < a.ny;
    const size_t n = (size_t)(in ? y : 0) * a.pitch + (in ? x : 0);
    const uint32_t cw = in ? a.cell[n] : 0u;
    const uint32_t type = update_type(cw);
    double part[4] = {0.0, 0.0, 0.0, 0.0};
    if (in && type != kSolid) {
        const size_t P = a.plane;
        // boundary velocity: the inlet profile, or a Neumann outlet's neighbour
        CT bx = type == kInlet ? (CT)a.uin[y] : CT(0), by = CT(0);
        if (BC && type == kOutletNeumann && (cw & kWordLeftLive)) {
            CT g[9];
#pragma unroll
            for (int i = 0; i < 9; ++i) g[i] = Cell::load(a.fin[(size_t)i * P + n - 1]);
            Cell::velocity(g, bx, by);
        }
        CT f[9];
        if (BC && (cw & kWordGeneral)) {
#pragma unroll
            for (int i = 0; i < 9; ++i)
                f[i] = Cell::load(a.fin[general_src(cw, i, x, y, y, a.ny, a.flags, P, a.pitch)]);
        } else {
#pragma unroll
            for (int i = 0; i < 9; ++i) {
                const bool wall = i > 0 && ((cw >> (i - 1)) & 1u);
                const size_t src = wall ? (size_t)kOpp[i] * P + n
                                        : (size_t)i * P + n - kCx[i] - (ptrdiff_t)kCy[i] * a.pitch;
                f[i] = Cell::load(a.fin[src]);
            }
        }
        double mass, ux, uy;
        Cell::update(f, type, bx, by, a, mass, ux, uy);
#pragma unroll
        for (int i = 0; i < 9; ++i) a.fout[(size_t)i * P + n] = Cell::store(f[i]);
        if (CHECK) check_terms(a, n, mass, ux, uy, part);
    }
    if (CHECK) {
        block_sum<4, 256>(part);
        if (threadIdx.x == 0 && threadIdx.y == 0) {
#pragma unroll
            for (int k = 0; k < 4; ++k) part_out[k] = part[k];
        }
    }
}

template <class Cell, bool CHECK, bool BC>
__global__ __launch_bounds__(256) void step_kernel(SweepArgs<typename Cell::T> a) {
    step_body<Cell, CHECK, BC>(
        a, blockIdx.x, blockIdx.y,
        CHECK ? a.partials + ((size_t)blockIdx.y * gridDim.x + blockIdx.x) * 4 : nullptr);
}

// One time step of many lattices: work item b is the 64 x 4 block
// blocks[b] (packed block row << 16 | block column) of lattice lat[b];
// lat[b] < 0 marks a padding item.
template <class Cell, bool BC>
__global__ __launch_bounds__(256) void step_batch_kernel(
    const SweepArgs<typename Cell::T> *__restrict__ args, const int32_t *__restrict__ lat,
    const int32_t *__restrict__ blocks) {
    const int l = lat[blockIdx.x];
    if (l < 0) return;
    const SweepArgs<typename Cell::T> a = args[l];
    const int t = blocks[blockIdx.x];
    step_body<Cell, false, BC>(a, t & 0xffff, t >> 16, nullptr);
}

// Temporal blocking.  Tile t = tiles[blockIdx.x] packs (tile row << 16 | tile
// column); the tile's cells are [tx*IW, tx*IW+IW) x [ty*IH, ty*IH+IH).
// Lane l of wave w owns region cells (l, w + c*NW), c = 0..CPT-1.  Two LDS
// copies of the region, interleaved by plane (plane i of copy b at index
// (2i + b) * PL): each step reads one copy and writes the other, with one
// barrier per step.  The step loop is unrolled by two so that the copy is a
// compile-time constant; each pull then reads a per-cell LDS byte address,
// computed once per launch, plus an immediate offset.  A cell's depth (its
// distance to the region edge; 0 for solid cells) bounds the steps it can
// take: it is advanced at step s exactly when depth >= s, and is a tile cell
// exactly when depth >= H.
template <class Cell, int RH, int H, int NT, bool CHECK, bool BC, bool HALT, bool PREV>
__device__ __forceinline__ void tb_body(const SweepArgs<typename Cell::T> &a, const int t,
                                        const int steps, double *part_out) {
    using T = typename Cell::T;
    using CT = typename Cell::CT;
    constexpr int RW = 64, IW = RW - 2 * H, IH = RH - 2 * H;
    constexpr int NW = NT / 64, CPT = RH / NW, PL = RW * RH;
    static_assert(RH % NW == 0, "region rows must split evenly over waves");
    static_assert((size_t)PL * sizeof(T) < 65536, "copy offset must fit an LDS immediate");
    extern __shared__ __align__(16) unsigned char lds_raw[];
    T *L = reinterpret_cast<T *>(lds_raw);

    const int ox = (t & 0xffff) * IW - H, oy = (t >> 16) * IH - H;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    RunGate<NT, HALT, PREV> gate;
    gate.read(a);  // beside the region's loads
    const int gx = ox + lane;
    const bool col_in = gx >= 0 && gx < a.nx;

    uint32_t cw[CPT];
    int depth[CPT];
    const T *src[CPT][9];  // LDS address of each pull in copy 0
    StoreBases<T, PL> dst[CPT];
    UinT<T> uin[CPT];      // inlet velocity of the thread's cells, read once per launch
    T v[CPT][9];
    size_t n[CPT];
    // The cell words of all the thread's cells are read first, then all their
    // populations, before the first LDS store, so that the HBM latencies
    // overlap; solid cells are not read.
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
        const int gy = oy + wave + c * NW;
        const bool in = col_in && gy >= 0 && gy < a.ny;
        n[c] = in ? (size_t)gy * a.pitch + gx : 0;
        cw[c] = in ? a.cell[n[c]] : 0u;
    }
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
        const int ry = wave + c * NW, gy = oy + ry;
        const bool live = cell_type(cw[c]) != kSolid;  // cells off the lattice read as solid
        depth[c] = live ? min(min(lane, RW - 1 - lane), min(ry, RH - 1 - ry)) : 0;
        uin[c] = cell_type(cw[c]) == kInlet ? a.uin[gy] : UinT<T>(0);
        if (live) {
            const T *p = a.fin + n[c];
#pragma unroll
            for (int i = 0; i < 9; ++i) v[c][i] = p[(size_t)i * a.plane];
        } else {
#pragma unroll
            for (int i = 0; i < 9; ++i) v[c][i] = Cell::store(CT(0));
        }
    }
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
        const int pos = (wave + c * NW) * RW + lane;
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            L[2 * i * PL + pos] = v[c][i];
            const bool wall = i > 0 && ((cw[c] >> (i - 1)) & 1u);
            const int e = wall ? 2 * kOpp[i] * PL + pos : 2 * i * PL + pos - kCy[i] * RW - kCx[i];
            src[c][i] = L + e;
        }
        dst[c].set(L, pos);
    }
    if (gate.ended(a)) return;
    __syncthreads();
    if (gate.ends_now(a)) return;

    double part[4] = {0.0, 0.0, 0.0, 0.0};
    // One step reading copy B and writing copy 1 - B; true when it was the last.
    auto step = [&](auto copy, const int s) -> bool {
        constexpr int B = decltype(copy)::value;
        const bool last = s == steps;
        const int need = last ? H : s;
#pragma unroll
        for (int c = 0; c < CPT; ++c) {
            if (depth[c] < need) continue;
            const int ry = wave + c * NW, gy = oy + ry, pos = ry * RW + lane;
            const uint32_t type = update_type(cw[c]);
            CT bx = type == kInlet ? (CT)uin[c] : CT(0), by = CT(0);
            if (BC && type == kOutletNeumann && (cw[c] & kWordLeftLive)) {
                CT g[9];
#pragma unroll
                for (int i = 0; i < 9; ++i) g[i] = Cell::load(L[(2 * i + B) * PL + pos - 1]);
                Cell::velocity(g, bx, by);
            }
            CT f[9];
            if (BC && (cw[c] & kWordGeneral)) {
#pragma unroll
                for (int i = 0; i < 9; ++i)
                    f[i] = Cell::load(
                        L[general_src(cw[c], i, lane, ry, gy, a.ny, a.flags, 2 * PL, RW) + B * PL]);
            } else {
#pragma unroll
                for (int i = 0; i < 9; ++i)
                    f[i] = Cell::load(src[c][i][B * PL]);
            }
            double mass, ux, uy;
            Cell::update(f, type, bx, by, a, mass, ux, uy);
            if (last) {
                const size_t n = (size_t)gy * a.pitch + gx;
#pragma unroll
                for (int i = 0; i < 9; ++i) a.fout[(size_t)i * a.plane + n] = Cell::store(f[i]);
                if (CHECK) check_terms(a, n, mass, ux, uy, part);
            } else {
#pragma unroll
                for (int i = 0; i < 9; ++i) dst[c].template put<1 - B>(i, Cell::store(f[i]));
            }
        }
        if (last) return true;
        __syncthreads();
        return false;
    };
    for (int s = 1; s <= steps; s += 2) {
        if (step(std::integral_constant<int, 0>{}, s)) break;
        if (step(std::integral_constant<int, 1>{}, s + 1)) break;
    }
    if (CHECK) {
        block_sum<4, NT>(part);
        if (threadIdx.x == 0) {
#pragma unroll
            for (int k = 0; k < 4; ++k) part_out[k] = part[k];
        }
    }
}

// Temporal blocking with one region copy, updated in place: at each step
// every thread first pulls the nine populations of each of its cells into
// registers, and after a barrier relaxes them and writes them back (two
// barriers per step).  Half the LDS of the two-copy form, so regions twice
// as tall fit (FP64 64 x 32: 147 KB).  Cells, depths and the order of the
// arithmetic are those of the two-copy form, so the results are the same
// bits.
template <class Cell, int RH, int H, int NT, bool CHECK, bool BC, bool HALT, bool PREV>
__device__ __forceinline__ void tb_body_inplace(const SweepArgs<typename Cell::T> &a,
                                                const int t, const int steps,
                                                double *part_out) {
    using T = typename Cell::T;
    using CT = typename Cell::CT;
    constexpr int RW = 64, IW = RW - 2 * H, IH = RH - 2 * H;
    constexpr int NW = NT / 64, CPT = RH / NW, PL = RW * RH;
    static_assert(RH % NW == 0, "region rows must split evenly over waves");
    extern __shared__ __align__(16) unsigned char lds_raw[];
    T *L = reinterpret_cast<T *>(lds_raw);

    const int ox = (t & 0xffff) * IW - H, oy = (t >> 16) * IH - H;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    RunGate<NT, HALT, PREV> gate;
    gate.read(a);  // beside the region's loads
    const int gx = ox + lane;
    const bool col_in = gx >= 0 && gx < a.nx;

    uint32_t cw[CPT];
    int depth[CPT];
    UinT<T> uin[CPT];  // inlet velocity of the thread's cells, read once per launch
    T v[CPT][9];
    size_t n[CPT];
    // cell words, then populations, then the LDS stores (as in the two-copy form)
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
        const int gy = oy + wave + c * NW;
        const bool in = col_in && gy >= 0 && gy < a.ny;
        n[c] = in ? (size_t)gy * a.pitch + gx : 0;
        cw[c] = in ? a.cell[n[c]] : 0u;
    }
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
        const int ry = wave + c * NW, gy = oy + ry;
        const bool live = cell_type(cw[c]) != kSolid;  // cells off the lattice read as solid
        depth[c] = live ? min(min(lane, RW - 1 - lane), min(ry, RH - 1 - ry)) : 0;
        uin[c] = cell_type(cw[c]) == kInlet ? a.uin[gy] : UinT<T>(0);
        if (live) {
            const T *p = a.fin + n[c];
#pragma unroll
            for (int i = 0; i < 9; ++i) v[c][i] = p[(size_t)i * a.plane];
        } else {
#pragma unroll
            for (int i = 0; i < 9; ++i) v[c][i] = Cell::store(CT(0));
        }
    }
#pragma unroll
    for (int c = 0; c < CPT; ++c)
#pragma unroll
        for (int i = 0; i < 9; ++i) L[i * PL + (wave + c * NW) * RW + lane] = v[c][i];
    if (gate.ended(a)) return;
    __syncthreads();
    if (gate.ends_now(a)) return;

    double part[4] = {0.0, 0.0, 0.0, 0.0};
    // Pulls of one cell (its nine populations after streaming, and for a
    // Neumann outlet the neighbour's velocity).
    auto pull = [&](const int c, CT (&f)[9], CT &bx, CT &by) {
        const int ry = wave + c * NW, gy = oy + ry, pos = ry * RW + lane;
        const uint32_t type = update_type(cw[c]);
        bx = type == kInlet ? (CT)uin[c] : CT(0);
        by = CT(0);
        if (BC && type == kOutletNeumann && (cw[c] & kWordLeftLive)) {
            CT g[9];
#pragma unroll
            for (int i = 0; i < 9; ++i) g[i] = Cell::load(L[i * PL + pos - 1]);
            Cell::velocity(g, bx, by);
        }
        if (BC && (cw[c] & kWordGeneral)) {
#pragma unroll
            for (int i = 0; i < 9; ++i)
                f[i] = Cell::load(L[general_src(cw[c], i, lane, ry, gy, a.ny, a.flags, PL, RW)]);
        } else {
#pragma unroll
            for (int i = 0; i < 9; ++i) {
                const bool wall = i > 0 && ((cw[c] >> (i - 1)) & 1u);
                f[i] = Cell::load(L[wall ? kOpp[i] * PL + pos : i * PL + pos - kCy[i] * RW - kCx[i]]);
            }
        }
    };
    for (int s = 1; s < steps; ++s) {
        // every read of the step, then a barrier, then the in-place writes
        CT f[CPT][9], bx[CPT], by[CPT];
#pragma unroll
        for (int c = 0; c < CPT; ++c)
            if (depth[c] >= s) pull(c, f[c], bx[c], by[c]);
        __syncthreads();
#pragma unroll
        for (int c = 0; c < CPT; ++c) {
            if (depth[c] < s) continue;
            double mass, ux, uy;
            Cell::update(f[c], update_type(cw[c]), bx[c], by[c], a, mass, ux, uy);
            const int pos = (wave + c * NW) * RW + lane;
#pragma unroll
            for (int i = 0; i < 9; ++i) L[i * PL + pos] = Cell::store(f[c][i]);
        }
        __syncthreads();
    }
    // The last step writes to HBM only, so each cell is pulled and updated in turn.
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
        if (depth[c] < H) continue;  // the tile cells
        CT f[9], bx, by;
        pull(c, f, bx, by);
        double mass, ux, uy;
        Cell::update(f, update_type(cw[c]), bx, by, a, mass, ux, uy);
        const size_t m = (size_t)(oy + wave + c * NW) * a.pitch + gx;
#pragma unroll
        for (int i = 0; i < 9; ++i) a.fout[(size_t)i * a.plane + m] = Cell::store(f[i]);
        if (CHECK) check_terms(a, m, mass, ux, uy, part);
    }
    if (CHECK) {
        block_sum<4, NT>(part);
        if (threadIdx.x == 0) {
#pragma unroll
            for (int k = 0; k < 4; ++k) part_out[k] = part[k];
        }
    }
}

// Temporal blocking with a compacted cell list.  On sparse geometries most
// lanes of a region row hold solid cells, so the dense form above issues
// every wave instruction for a few useful lanes.  Here, after the region is
// in LDS, the workgroup lists its non-solid cells (LDS position and cell
// word) ordered by class k = min(depth, H), largest first, where depth is
// the distance to the region edge: a cell can be advanced at step s exactly
// when depth >= s, and is a tile cell exactly when depth >= H.  So at every
// step the cells to update are a prefix of the list, and consecutive lanes
// take consecutive entries.  Within a class, entries keep row-major order.
// Each update reads the same nine values as the dense form, so the results
// are the same bits.  LDS: the two region copies, interleaved by plane as in
// the dense form, then PL list words.
template <class Cell, int RH, int H, int NT, bool CHECK, bool BC, bool HALT, bool PREV>
__device__ __forceinline__ void tb_body_compact(const SweepArgs<typename Cell::T> &a, const int t,
                                                const int steps, double *part_out) {
    using T = typename Cell::T;
    using CT = typename Cell::CT;
    constexpr int RW = 64, IW = RW - 2 * H, IH = RH - 2 * H;
    constexpr int NW = NT / 64, CPT = RH / NW, PL = RW * RH;
    static_assert(RH % NW == 0, "region rows must split evenly over waves");
    static_assert(PL <= 65536 && RH <= 64, "list entries pack the position in 16 bits");
    extern __shared__ __align__(16) unsigned char lds_raw[];
    T *L = reinterpret_cast<T *>(lds_raw);
    uint32_t *list = reinterpret_cast<uint32_t *>(lds_raw + (size_t)2 * 9 * PL * sizeof(T));
    __shared__ int row_off[RH][H];  // per row and class: count, then offset
    __shared__ int cls_total[H + 1];
    __shared__ int cls_base[H + 2];

    const int ox = (t & 0xffff) * IW - H, oy = (t >> 16) * IH - H;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    RunGate<NT, HALT, PREV> gate;
    gate.read(a);  // beside the region's loads
    const int gx = ox + lane;
    const bool col_in = gx >= 0 && gx < a.nx;
    const uint64_t below = (1ull << lane) - 1ull;

    int cls[CPT];
    uint32_t cw[CPT];
    size_t n[CPT];
    T v[CPT][9];
    // Cell words first, then populations, then the LDS stores, so that the
    // HBM latencies overlap; solid cells are not read.
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
        const int gy = oy + wave + c * NW;
        const bool in = col_in && gy >= 0 && gy < a.ny;
        n[c] = in ? (size_t)gy * a.pitch + gx : 0;
        cw[c] = in ? a.cell[n[c]] : 0u;
    }
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
        if (cell_type(cw[c]) != kSolid) {  // cells off the lattice read as solid
            const T *p = a.fin + n[c];
#pragma unroll
            for (int i = 0; i < 9; ++i) v[c][i] = p[(size_t)i * a.plane];
        } else {
#pragma unroll
            for (int i = 0; i < 9; ++i) v[c][i] = Cell::store(CT(0));
        }
    }
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
        const int ry = wave + c * NW;
        const bool live = cell_type(cw[c]) != kSolid;
#pragma unroll
        for (int i = 0; i < 9; ++i) L[2 * i * PL + ry * RW + lane] = v[c][i];
        const int depth = min(min(lane, RW - 1 - lane), min(ry, RH - 1 - ry));
        cls[c] = live ? min(depth, H) : 0;
#pragma unroll
        for (int k = 1; k <= H; ++k) {
            const uint64_t m = __ballot(cls[c] == k);
            if (lane == 0) row_off[ry][k - 1] = __popcll(m);
        }
    }
    if (gate.ended(a)) return;
    __syncthreads();
    if (gate.ends_now(a)) return;
    if (threadIdx.x < H) {  // one thread per class: exclusive scan over rows
        const int k = threadIdx.x;
        int run = 0;
        for (int r = 0; r < RH; ++r) {
            const int v = row_off[r][k];
            row_off[r][k] = run;
            run += v;
        }
        cls_total[k + 1] = run;
    }
    __syncthreads();
    if (threadIdx.x == 0) {  // classes in decreasing order; cls_base[k] = entries of class > k
        int run = 0;
        cls_base[H + 1] = 0;
        for (int k = H; k >= 1; --k) {
            cls_base[k] = run;
            run += cls_total[k];
        }
        cls_base[0] = run;
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
        const int ry = wave + c * NW;
#pragma unroll
        for (int k = 1; k <= H; ++k) {
            const uint64_t m = __ballot(cls[c] == k);
            if (cls[c] == k)
                list[cls_base[k] + row_off[ry][k - 1] + __popcll(m & below)] =
                    (cw[c] << 16) | (uint32_t)(ry * RW + lane);
        }
    }
    __syncthreads();
    const int n_all = cls_base[0];
    uint32_t ent[CPT];
    const T *src[CPT][9];  // LDS address of each pull of the thread's entries in copy 0
    StoreBases<T, PL> dst[CPT];
    UinT<T> uin[CPT];      // inlet velocity of the thread's entries, read once per launch
#pragma unroll
    for (int m = 0; m < CPT; ++m) {
        const int j = threadIdx.x + m * NT;
        ent[m] = j < n_all ? list[j] : 0u;
        const uint32_t c = ent[m] >> 16;
        const int pos = (int)(ent[m] & 0xffffu);
        dst[m].set(L, pos);
        uin[m] = (j < n_all && cell_type(c) == kInlet) ? a.uin[oy + pos / RW] : UinT<T>(0);
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            const bool wall = i > 0 && ((c >> (i - 1)) & 1u);
            const int e = wall ? 2 * kOpp[i] * PL + pos : 2 * i * PL + pos - kCy[i] * RW - kCx[i];
            src[m][i] = L + e;
        }
    }

    double part[4] = {0.0, 0.0, 0.0, 0.0};
    // One step reading copy B and writing copy 1 - B; true when it was the last.
    auto step = [&](auto copy, const int s) -> bool {
        constexpr int B = decltype(copy)::value;
        const bool last = s == steps;
        // cells of class >= s, or the tile cells (class H) at the last step
        const int n_s = last ? cls_base[H] + cls_total[H] : cls_base[s] + cls_total[s];
#pragma unroll
        for (int m = 0; m < CPT; ++m) {
            if (threadIdx.x + m * NT >= n_s) continue;
            const uint32_t c = ent[m] >> 16;
            const int pos = (int)(ent[m] & 0xffffu);
            const int ry = pos / RW, lx = pos % RW;
            const uint32_t type = update_type(c);
            const int gy = oy + ry;
            CT bx = type == kInlet ? (CT)uin[m] : CT(0), by = CT(0);
            if (BC && type == kOutletNeumann && (c & kWordLeftLive)) {
                CT g[9];
#pragma unroll
                for (int i = 0; i < 9; ++i) g[i] = Cell::load(L[(2 * i + B) * PL + pos - 1]);
                Cell::velocity(g, bx, by);
            }
            CT f[9];
            if (BC && (c & kWordGeneral)) {
#pragma unroll
                for (int i = 0; i < 9; ++i)
                    f[i] = Cell::load(
                        L[general_src(c, i, lx, ry, gy, a.ny, a.flags, 2 * PL, RW) + B * PL]);
            } else {
#pragma unroll
                for (int i = 0; i < 9; ++i) f[i] = Cell::load(src[m][i][B * PL]);
            }
            double mass, ux, uy;
            Cell::update(f, type, bx, by, a, mass, ux, uy);
            if (last) {
                const size_t n = (size_t)gy * a.pitch + (ox + lx);
#pragma unroll
                for (int i = 0; i < 9; ++i) a.fout[(size_t)i * a.plane + n] = Cell::store(f[i]);
                if (CHECK) check_terms(a, n, mass, ux, uy, part);
            } else {
#pragma unroll
                for (int i = 0; i < 9; ++i) dst[m].template put<1 - B>(i, Cell::store(f[i]));
            }
        }
        if (last) return true;
        __syncthreads();
        return false;
    };
    for (int s = 1; s <= steps; s += 2) {
        if (step(std::integral_constant<int, 0>{}, s)) break;
        if (step(std::integral_constant<int, 1>{}, s + 1)) break;
    }
    if (CHECK) {
        block_sum<4, NT>(part);
        if (threadIdx.x == 0) {
#pragma unroll
            for (int k = 0; k < 4; ++k) part_out[k] = part[k];
        }
    }
}

// One region shape: rows x 64 cells, halo H, body KIND (TbKind).  HALT: the
// launch may belong to a queued run that has already ended (SweepArgs::stop);
// PREV: it is the first launch of a queued interval that decides the
// interval before it (SweepArgs::prev; never a check launch).
template <class Cell, int RH, int H, int NT, int KIND, bool CHECK, bool BC, bool HALT,
          bool PREV>
__device__ __forceinline__ void tb_dispatch(const SweepArgs<typename Cell::T> &a, const int t,
                                            const int steps, double *part_out) {
    if constexpr (KIND == kTbCompact)
        tb_body_compact<Cell, RH, H, NT, CHECK, BC, HALT, PREV>(a, t, steps, part_out);
    else if constexpr (KIND == kTbInPlace)
        tb_body_inplace<Cell, RH, H, NT, CHECK, BC, HALT, PREV>(a, t, steps, part_out);
    else
        tb_body<Cell, RH, H, NT, CHECK, BC, HALT, PREV>(a, t, steps, part_out);
}

// The tile list, the stop flag's lane copies (SweepArgs::stop) and the step
// count come first, so that they arrive preloaded in scalar registers: the
// tile's index and the flag are then requested at once, beside the remaining
// arguments, instead of after them.
template <class Cell, int RH, int H, int NT, int KIND, bool CHECK, bool BC, bool PREV>
__global__ __launch_bounds__(NT) void tb_kernel(const int32_t *__restrict__ tiles,
                                                const int *__restrict__ stop, int steps,
                                                SweepArgs<typename Cell::T> args) {
    static_assert(!(CHECK && PREV), "a check launch does not decide the interval before it");
    SweepArgs<typename Cell::T> a = args;
    a.stop = stop;
    tb_dispatch<Cell, RH, H, NT, KIND, CHECK, BC, true, PREV>(
        a, tiles[blockIdx.x], steps, CHECK ? a.partials + (size_t)blockIdx.x * 4 : nullptr);
}

// Many lattices in one launch: work item b is tile tiles[b] of lattice
// lat[b], whose arguments are args[lat[b]]; lat[b] < 0 marks a padding item
// (the whole workgroup leaves at once, before any barrier).
template <class Cell, int RH, int H, int NT, int KIND, bool BC>
__global__ __launch_bounds__(NT) void tb_batch_kernel(
    const SweepArgs<typename Cell::T> *__restrict__ args, const int32_t *__restrict__ lat,
    const int32_t *__restrict__ tiles, int steps) {
    const int l = lat[blockIdx.x];
    if (l < 0) return;
    const SweepArgs<typename Cell::T> a = args[l];
    tb_dispatch<Cell, RH, H, NT, KIND, false, BC, false, false>(a, tiles[blockIdx.x], steps,
                                                                 nullptr);
}

// Dynamic LDS of one region shape.
template <typename T, int RH, int KIND>
constexpr size_t tb_lds_bytes() {
    return (size_t)(KIND == kTbInPlace ? 1 : 2) * 9 * 64 * RH * sizeof(T) +
           (KIND == kTbCompact ? (size_t)64 * RH * sizeof(uint32_t) : 0);
}

// Host-side launch helpers shared by the per-precision units.
template <class Cell>
hipError_t launch_step(const SweepArgs<typename Cell::T> &a, bool check, hipStream_t s) {
    const dim3 g((unsigned)((a.nx + 63) / 64), (unsigned)((a.ny + 3) / 4)), b(64, 4);
    const bool bc = a.flags != 0;
    if (check && bc)
        hipLaunchKernelGGL((step_kernel<Cell, true, true>), g, b, 0, s, a);
    else if (check)
        hipLaunchKernelGGL((step_kernel<Cell, true, false>), g, b, 0, s, a);
    else if (bc)
        hipLaunchKernelGGL((step_kernel<Cell, false, true>), g, b, 0, s, a);
    else
        hipLaunchKernelGGL((step_kernel<Cell, false, false>), g, b, 0, s, a);
    return hipGetLastError();
}

// Raise a kernel's dynamic LDS limit; `done` is the caller's per-kernel flag.
inline hipError_t set_lds(const void *k, size_t lds, bool &done) {
    if (done) return hipSuccess;
    const hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e == hipSuccess) done = true;
    return e;
}

template <class Cell, int RH, int H, int NT, int KIND, bool CHECK, bool BC, bool PREV = false>
hipError_t launch_tb_one(const SweepArgs<typename Cell::T> &a, const int32_t *tiles, int n_tiles,
                         int steps, hipStream_t s) {
    const size_t lds = tb_lds_bytes<typename Cell::T, RH, KIND>();
    auto k = tb_kernel<Cell, RH, H, NT, KIND, CHECK, BC, PREV>;
    static bool configured = false;  // one flag per kernel instantiation
    const hipError_t e = set_lds((const void *)k, lds, configured);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k, dim3((unsigned)n_tiles), dim3(NT), lds, s, tiles, a.stop, steps, a);
    return hipGetLastError();
}

template <class Cell, int RH, int H, int NT, int KIND>
hipError_t launch_tb(const SweepArgs<typename Cell::T> &a, const int32_t *tiles, int n_tiles,
                     int steps, bool check, hipStream_t s) {
    if (n_tiles <= 0 || steps <= 0) return hipSuccess;
    if (steps > H) return hipErrorInvalidValue;
    const bool bc = a.flags != 0;
    if (a.prev) {
        if (check || n_tiles > kDeferMaxPartials) return hipErrorInvalidValue;
        if (bc)
            return launch_tb_one<Cell, RH, H, NT, KIND, false, true, true>(a, tiles, n_tiles,
                                                                           steps, s);
        return launch_tb_one<Cell, RH, H, NT, KIND, false, false, true>(a, tiles, n_tiles, steps,
                                                                        s);
    }
    if (check && bc)
        return launch_tb_one<Cell, RH, H, NT, KIND, true, true>(a, tiles, n_tiles, steps, s);
    if (check)
        return launch_tb_one<Cell, RH, H, NT, KIND, true, false>(a, tiles, n_tiles, steps, s);
    if (bc)
        return launch_tb_one<Cell, RH, H, NT, KIND, false, true>(a, tiles, n_tiles, steps, s);
    return launch_tb_one<Cell, RH, H, NT, KIND, false, false>(a, tiles, n_tiles, steps, s);
}

template <class Cell, int RH, int H, int NT, int KIND, bool BC>
hipError_t launch_tb_batch_one(const SweepArgs<typename Cell::T> *args, const int32_t *lat,
                               const int32_t *tiles, int n_items, int steps, hipStream_t s) {
    const size_t lds = tb_lds_bytes<typename Cell::T, RH, KIND>();
    auto k = tb_batch_kernel<Cell, RH, H, NT, KIND, BC>;
    static bool configured = false;  // one flag per kernel instantiation; set also on an
                                     // empty call, so that it can precede a graph capture
    const hipError_t e = set_lds((const void *)k, lds, configured);
    if (e != hipSuccess) return e;
    if (n_items <= 0 || steps <= 0) return hipSuccess;
    hipLaunchKernelGGL(k, dim3((unsigned)n_items), dim3(NT), lds, s, args, lat, tiles, steps);
    return hipGetLastError();
}

template <class Cell, int RH, int H, int NT, int KIND>
hipError_t launch_tb_batch(const SweepArgs<typename Cell::T> *args, const int32_t *lat,
                           const int32_t *tiles, int n_items, int steps, bool bc, hipStream_t s) {
    if (steps > H) return hipErrorInvalidValue;
    if (bc)
        return launch_tb_batch_one<Cell, RH, H, NT, KIND, true>(args, lat, tiles, n_items,
                                                                       steps, s);
    return launch_tb_batch_one<Cell, RH, H, NT, KIND, false>(args, lat, tiles, n_items,
                                                                    steps, s);
}

template <class Cell>
hipError_t launch_step_batch(const SweepArgs<typename Cell::T> *args, const int32_t *lat,
                             const int32_t *blocks, int n_items, bool bc, hipStream_t s) {
    if (n_items <= 0) return hipSuccess;
    if (bc)
        hipLaunchKernelGGL((step_batch_kernel<Cell, true>), dim3((unsigned)n_items), dim3(64, 4),
                           0, s, args, lat, blocks);
    else
        hipLaunchKernelGGL((step_batch_kernel<Cell, false>), dim3((unsigned)n_items), dim3(64, 4),
                           0, s, args, lat, blocks);
    return hipGetLastError();
}

// Run-time choice among the compiled region shapes of the storage type.
template <class Cell, int V = 0>
hipError_t launch_tb_variant(const SweepArgs<typename Cell::T> &a, const int32_t *tiles,
                             int n_tiles, int steps, bool check, int variant, hipStream_t s) {
    using T = typename Cell::T;
    if constexpr (V < TbVariants<T>::count) {
        if (variant == V)
            return launch_tb<Cell, TbVariants<T>::v[V].rows, TbVariants<T>::v[V].halo,
                             kTbThreads, TbVariants<T>::v[V].kind>(a, tiles, n_tiles,
                                                                            steps, check, s);
        return launch_tb_variant<Cell, V + 1>(a, tiles, n_tiles, steps, check, variant, s);
    } else {
        return hipErrorInvalidValue;
    }
}

template <class Cell, int V = 0>
hipError_t launch_tb_batch_variant(const SweepArgs<typename Cell::T> *args, const int32_t *lat,
                                   const int32_t *tiles, int n_items, int steps, int variant,
                                   bool bc, hipStream_t s) {
    using T = typename Cell::T;
    if constexpr (V < TbVariants<T>::count) {
        if (variant == V)
            return launch_tb_batch<Cell, TbVariants<T>::v[V].rows, TbVariants<T>::v[V].halo,
                                   kTbThreads, TbVariants<T>::v[V].kind>(
                args, lat, tiles, n_items, steps, bc, s);
        return launch_tb_batch_variant<Cell, V + 1>(args, lat, tiles, n_items, steps, variant,
                                                    bc, s);
    } else {
        return hipErrorInvalidValue;
    }
}

}  // namespace sweep
}  // namespace lbm
