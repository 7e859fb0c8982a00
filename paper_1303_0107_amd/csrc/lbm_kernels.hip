// Single-precision sweep kernels and the precision-independent kernels (cell
// words, exchange step) of the D2Q9 lattice-Boltzmann shape-optimisation path
// for gfx950 (MI355X).  The double-precision sweep lives in lbm_f64.hip.
// Wang, Fan & Luo, "Lattice Boltzmann method for shape optimization of fluid
// distributor": Sec. 2.1 (LBE, equilibrium, moments),
// Sec. 2.2 (exchange criteria, Eqs. 5-6), Sec. 3.3 (boundary conditions),
// Sec. 4.2 (Eqs. 9-11), Eq. 4 (pressure).
//
// Memory layout (see lbm_internal.h):
//   populations  nine planes of ny rows x pitch columns, pitch a multiple of
//                64 so that every wavefront row segment is 64 consecutive
//                elements.  Single precision stores the offset d_i = f_i - w_i
//                of the post-collision population (about to stream), which
//                keeps the relative precision of the small deviations from
//                rest; double precision stores f_i itself.
//   cell words   uint16 per cell: bits 0..7 flag a wall on the pull link of
//                population 1..8 (source solid or outside the lattice),
//                bits 8..9 the cell type.
//   two population buffers, read one / write the other each step.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <stdint.h>

#include <cstring>

#include "lbm_boundary.h"
#include "lbm_internal.h"
#include "lbm_keys.h"
#include "lbm_sweep.h"

namespace lbm {

// D2Q9 numbering of Sec. 2.1.
__device__ constexpr int kCx[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
__device__ constexpr int kCy[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
__device__ constexpr int kOpp[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};

template <typename T>
__device__ __forceinline__ T wgt(int i) {
    return i == 0 ? T(4) / T(9) : (i < 5 ? T(1) / T(9) : T(1) / T(36));
}

// Moments of nine offsets with the mirror-symmetric pairing of the sweep:
// density offset, x and y momentum.
__device__ __forceinline__ void moments_sym(const double (&d)[9], double &dr,
                                            double &jx, double &jy) {
    dr = ((d[0] + (d[1] + d[3])) + (d[2] + d[4])) + ((d[5] + d[8]) + (d[6] + d[7]));
    jx = (d[1] + (d[5] + d[8])) - (d[3] + (d[6] + d[7]));
    jy = (d[2] + (d[5] + d[6])) - (d[4] + (d[8] + d[7]));
}

// Density and velocity (Eq. 2) of the stored offsets of cell n (pitched), in
// double: the macroscopic export and the exchange-step keys both use this.
template <typename S>
struct OffsetMoments {
    using T = S;
    __device__ static __forceinline__ void at(const S *f, size_t plane, size_t n, double &rho,
                                              double &ux, double &uy) {
        double d[9];
#pragma unroll
        for (int i = 0; i < 9; ++i) d[i] = Sto<S>::to_d(f[(size_t)i * plane + n]);
        double dr, jx, jy;
        moments_sym(d, dr, jx, jy);
        rho = 1.0 + dr;
        ux = jx / rho;
        uy = jy / rho;
    }
};

// ---------------------------------------------------------------------------
// Wavefront / block reductions of NV doubles (fixed order: results do not
// depend on scheduling).
template <int NV>
__device__ __forceinline__ void wave_sum(double (&v)[NV]) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
#pragma unroll
        for (int k = 0; k < NV; ++k) v[k] += __shfl_xor(v[k], off, 64);
}

// Sum over a block of `nthreads` (multiple of 64, <= 1024); the result is
// valid in thread 0.
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], int tid,
                                          int nthreads) {
    __shared__ double red[16][NV];
    wave_sum<NV>(v);
    const int wave = tid >> 6, lane = tid & 63;
    if (lane == 0)
#pragma unroll
        for (int k = 0; k < NV; ++k) red[wave][k] = v[k];
    __syncthreads();
    if (tid == 0) {
        const int nw = nthreads >> 6;
        for (int w = 1; w < nw; ++w)
#pragma unroll
            for (int k = 0; k < NV; ++k) v[k] += red[w][k];
    }
}

// ---------------------------------------------------------------------------
// One cell of one time step on offsets d_i = f_i - w_i stored as T (float,
// or 16-bit for the reduced-storage forms), arithmetic in CT, velocity
// polynomials in PT (all forms: float).  The relaxation restores exact mass
// and momentum conservation after rounding (see update); without that, the
// rounded weights bias every step the same way and float arithmetic, not
// the storage, dominated the error of steady fields.  Zou-He closure on inlet
// (velocity u_in, unknowns 1, 5, 8) and outlet cells (density rho_out, zero
// transverse velocity, unknowns 3, 6, 7), moments (Eq. 2), BGK relaxation
// (Eq. 1) to the equilibrium of Sec. 2.1 written for offsets:
// feq_i - w_i = w_i (drho + rho (3 c.u + 4.5 (c.u)^2 - 1.5 u.u)).  Every sum
// pairs the populations that a reflection y -> -y exchanges (2<->4, 5<->8,
// 6<->7) and every product maps to itself or its exact negative under it, so
// on a mirror-symmetric lattice the computed flow is mirror-symmetric bit for
// bit.  Multiply-adds are fused only inside one expression, as written, so
// every kernel that inlines this function rounds identically.
// Reciprocal for the per-cell arithmetic: in float the hardware reciprocal
// refined by one Newton step, r + r (1 - x r) (the raw estimate's error has
// a sign bias that the flux split between outlets integrates); in double
// the division.  The same in every kernel.
__device__ __forceinline__ float recip(float x) {
    const float r = __builtin_amdgcn_rcpf(x);
    return __builtin_fmaf(__builtin_fmaf(-x, r, 1.0f), r, r);
}
__device__ __forceinline__ double recip(double x) { return 1.0 / x; }

template <typename Storage, typename Arith, typename Poly>
struct OffsetCell {
    using T = Storage;
    using CT = Arith;
    using PT = Poly;
    __device__ static __forceinline__ CT load(T v) { return (CT)Sto<T>::to_d(v); }
    __device__ static __forceinline__ CT load_f(T v) { return (CT)Sto<T>::to_f(v); }
    __device__ static __forceinline__ T store(CT v) {
        if constexpr (sizeof(CT) == 8)
            return Sto<T>::from_d((double)v);
        else
            return Sto<T>::from_f((float)v);
    }
    // Velocity (Eq. 2) of a stored offset set, with the update's pairing.
    __device__ static __forceinline__ void velocity(const CT (&d)[9], CT &ux, CT &uy) {
        const CT dr = ((d[0] + (d[1] + d[3])) + (d[2] + d[4])) + ((d[5] + d[8]) + (d[6] + d[7]));
        const CT jx = (d[1] + (d[5] + d[8])) - (d[3] + (d[6] + d[7]));
        const CT jy = (d[2] + (d[5] + d[6])) - (d[4] + (d[8] + d[7]));
        const CT ir = recip(CT(1) + dr);
        ux = jx * ir;
        uy = jy * ir;
    }
    // (bx, by): the inlet velocity (inlet cells) or the velocity a Neumann
    // outlet imposes (that of its x-1 neighbour's stored state).
    __device__ static __forceinline__ void update(CT (&d)[9], uint32_t type, CT bx, CT by,
                                                  const SweepArgs<T> &a, double &mass,
                                                  double &ux_out, double &uy_out) {
#pragma clang fp contract(on)
        if (type == kFluid) {
            // no closure (the common case, tested first)
        } else if (type == kInlet) {
            const CT s = (d[0] + (d[2] + d[4])) + CT(2) * (d[3] + (d[6] + d[7]));
            const CT dr = (s + bx) * recip(CT(1) - bx);
            const CT ru = (CT(1) + dr) * bx;
            const CT h = CT(0.5) * (d[2] - d[4]);
            d[1] = d[3] + (CT(2) / CT(3)) * ru;
            d[5] = d[7] - h + (CT(1) / CT(6)) * ru;
            d[8] = d[6] + h + (CT(1) / CT(6)) * ru;
        } else if (type == kOutlet) {
            const CT s = (d[0] + (d[2] + d[4])) + CT(2) * (d[1] + (d[5] + d[8]));
            const CT uo = (s + (CT)a.one_minus_rho_out) * recip((CT)a.rho_out);
            const CT ru = (CT)a.rho_out * uo;
            const CT h = CT(0.5) * (d[2] - d[4]);
            d[3] = d[1] - (CT(2) / CT(3)) * ru;
            d[7] = d[5] + h - (CT(1) / CT(6)) * ru;
            d[6] = d[8] - h - (CT(1) / CT(6)) * ru;
        } else if (type == kOutletNeumann) {
            // rho = (1 + s) / (1 + ux): offsets of the Zou-He velocity closure
            const CT s = (d[0] + (d[2] + d[4])) + CT(2) * (d[1] + (d[5] + d[8]));
            const CT dr = (s - bx) * recip(CT(1) + bx);
            const CT ru = (CT(1) + dr) * bx, rv = (CT(1) + dr) * by;
            const CT h = CT(0.5) * (d[2] - d[4]);
            d[3] = d[1] - (CT(2) / CT(3)) * ru;
            d[7] = d[5] + h - (CT(1) / CT(6)) * ru - CT(0.5) * rv;
            d[6] = d[8] - h - (CT(1) / CT(6)) * ru + CT(0.5) * rv;
        }
        const CT dr = ((d[0] + (d[1] + d[3])) + (d[2] + d[4])) + ((d[5] + d[8]) + (d[6] + d[7]));
        const CT rho = CT(1) + dr;
        const CT jx = (d[1] + (d[5] + d[8])) - (d[3] + (d[6] + d[7]));
        const CT jy = (d[2] + (d[5] + d[6])) - (d[4] + (d[8] + d[7]));
        const CT ir = recip(rho);
        const CT ux = jx * ir, uy = jy * ir;
        const CT om = (CT)a.omega;
        // Opposite directions i, opp(i) have c.u = +-cu: their equilibrium
        // offsets share the even part A = 4.5 cu^2 - 1.5 u.u and differ in the
        // sign of the odd part B = 3 cu.
        const PT pux = (PT)ux, puy = (PT)uy;
        const PT puu15 = PT(1.5) * (pux * pux + puy * puy);
        // With the weights rounded (to float), the equilibrium's mass and
        // momentum differ from dr and (jx, jy) by ~1e-8 relative, every step,
        // with a fixed sign: a bias that the flow's slowest mode accumulates
        // over thousands of steps (a steady-state error ~1e-4).  So the
        // increments t_i = e_i - d_i toward equilibrium are corrected to
        // conserve exactly before the relaxation: the (1,3) and (2,4) pairs
        // take the momentum defects, t_0 the mass defect.  Each population
        // then relaxes as d_i + om t_i in one multiply-add.  Every sum is in
        // mirror-symmetric order, so a y-reflection maps each increment onto
        // its mirror image bit for bit.
        CT t[9];
        // A + B = (4.5 cu + 3) cu - 1.5 u.u and A - B = (4.5 cu - 3) cu - 1.5 u.u,
        // two multiply-adds each.
        auto incr_pair = [&](int i, int j, PT cu, CT w) {
            const PT hp = PT(4.5) * cu + PT(3), hm = PT(4.5) * cu - PT(3);
            const PT ApB = hp * cu - puu15, AmB = hm * cu - puu15;
            t[i] = w * (dr + rho * (CT)ApB) - d[i];
            t[j] = w * (dr + rho * (CT)AmB) - d[j];
        };
        const CT w1 = CT(1) / CT(9), w5 = CT(1) / CT(36);
        incr_pair(1, 3, pux, w1);
        incr_pair(2, 4, puy, w1);
        incr_pair(5, 7, pux + puy, w5);
        incr_pair(6, 8, puy - pux, w5);
        const CT mx = (t[1] - t[3]) + ((t[5] - t[7]) + (t[8] - t[6]));
        const CT my = (t[2] - t[4]) + ((t[5] - t[8]) + (t[6] - t[7]));
        t[1] = t[1] - CT(0.5) * mx;
        t[3] = t[3] + CT(0.5) * mx;
        t[2] = t[2] - CT(0.5) * my;
        t[4] = t[4] + CT(0.5) * my;
        t[0] = -(((t[1] + t[3]) + (t[2] + t[4])) + ((t[5] + t[8]) + (t[6] + t[7])));
#pragma unroll
        for (int i = 0; i < 9; ++i) d[i] = d[i] + om * t[i];
        mass = 1.0 + (double)dr;
        ux_out = (double)ux;
        uy_out = (double)uy;
    }
};

using F32Cell = OffsetCell<float, ArithT<float>, float>;
using H16Cell = OffsetCell<h16, ArithT<h16>, float>;
using BF16Cell = OffsetCell<bf16, ArithT<bf16>, float>;

// Sum `count` groups of NV doubles in a fixed order (one block of 256).
template <int NV>
__global__ __launch_bounds__(256) void finalize_kernel(const double *partials,
                                                       int64_t count,
                                                       double *out) {
    double v[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) v[k] = 0.0;
    for (int64_t j = threadIdx.x; j < count; j += 256)
#pragma unroll
        for (int k = 0; k < NV; ++k) v[k] += partials[j * NV + k];
    block_sum<NV>(v, threadIdx.x, 256);
    if (threadIdx.x == 0)
#pragma unroll
        for (int k = 0; k < NV; ++k) out[k] = v[k];
}

// The finalize step of one check interval of a queued run (see RunControl).
__global__ __launch_bounds__(256) void finalize_check_kernel(const double *partials,
                                                             int64_t count, RunControl *ctl,
                                                             int j, double tol) {
    if (ctl->stop) return;  // the run already ended: same value for every thread
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    for (int64_t i = threadIdx.x; i < count; i += 256)
#pragma unroll
        for (int k = 0; k < 4; ++k) v[k] += partials[i * 4 + k];
    block_sum<4>(v, threadIdx.x, 256);
    if (threadIdx.x == 0)
        sweep::record_interval(ctl, j, v, sweep::interval_stop(v, tol), ctl->stop_lanes[0],
                               ctl->stop_lanes[1]);
}

// ---------------------------------------------------------------------------
// Moments of the stored state (collision conserves rho and rho u, so these
// equal the moments of the state it was relaxed from).  Optional outputs:
// double rho/ux/uy in logical layout (y*nx + x; zero on solid cells), and
// the u_prev planes (pitched, type T).
template <typename T>
__global__ __launch_bounds__(256) void macro_kernel(MacroArgs<T> a) {
    const int x = blockIdx.x * 64 + threadIdx.x;
    const int y = blockIdx.y * 4 + threadIdx.y;
    if (x >= a.nx || y >= a.ny) return;
    const size_t n = (size_t)y * a.pitch + x;
    const size_t l = (size_t)y * a.nx + x;
    const bool solid = cell_type(a.cell[n]) == kSolid;
    double rho = 0.0, ux = 0.0, uy = 0.0;
    if (!solid) OffsetMoments<T>::at(a.f, a.plane, n, rho, ux, uy);
    if (a.rho) {
        a.rho[l] = rho;
        a.ux[l] = ux;
        a.uy[l] = uy;
    }
    if (a.uprev) {
        a.uprev[n] = ux;
        a.uprev[a.plane + n] = uy;
    }
}

// Per-block sum of rho over non-solid cells of the stored state.
template <typename T>
__global__ __launch_bounds__(256) void mass_kernel(MacroArgs<T> a,
                                                   double *partials) {
    const int x = blockIdx.x * 64 + threadIdx.x;
    const int y = blockIdx.y * 4 + threadIdx.y;
    double v[1] = {0.0};
    if (x < a.nx && y < a.ny) {
        const size_t n = (size_t)y * a.pitch + x;
        if (cell_type(a.cell[n]) != kSolid) {
            double d[9], dr, jx, jy;
#pragma unroll
            for (int i = 0; i < 9; ++i) d[i] = Sto<T>::to_d(a.f[(size_t)i * a.plane + n]);
            moments_sym(d, dr, jx, jy);
            v[0] = 1.0 + dr;
        }
    }
    const int tid = threadIdx.y * 64 + threadIdx.x;
    block_sum<1>(v, tid, 256);
    if (tid == 0) partials[(size_t)blockIdx.y * gridDim.x + blockIdx.x] = v[0];
}

// Boundary sums (Sec. 4.2) in increasing y: workgroup k < n_out sums rho u_x
// and rho over outlet k's rows y0..y1 (column nx-1); workgroup n_out sums
// over the inlet cells of column 0 and the density over all outlet cells.  out:
// [flow_0..flow_{n-1}, rho_0..rho_{n-1}, flow_in, rho_in, count_in,
//  count_out, rho_out]
template <typename T>
__global__ __launch_bounds__(kBoundaryThreads) void boundary_kernel(MacroArgs<T> a,
                                                                    const int32_t *out_y0,
                                                                    const int32_t *out_y1,
                                                                    int n_out, double *out) {
    // Workgroup k < n_out: outlet k, one wave (the others leave), its rows
    // read 64 at once; workgroup n_out: the inlet and all outlet cells
    // (boundary_ends).  The sums take the rows in increasing y, one row at a
    // time, so every sum has the order of a sequential loop.
    const int k = blockIdx.x, lane = threadIdx.x;
    auto moments = [&](size_t n, double &rho, double &jx) {
        double d[9];
#pragma unroll
        for (int i = 0; i < 9; ++i) d[i] = Sto<T>::to_d(a.f[(size_t)i * a.plane + n]);
        double dr, jy;
        moments_sym(d, dr, jx, jy);
        rho = 1.0 + dr;
    };
    if (k < n_out) {
        if (threadIdx.x >= 64) return;  // one wave per outlet
        const int y0 = out_y0[k], y1 = out_y1[k];
        double fl = 0.0, rs = 0.0;
        for (int c = y0; c <= y1; c += 64) {
            double r = 0.0, j = 0.0;
            if (c + lane <= y1) moments((size_t)(c + lane) * a.pitch + (a.nx - 1), r, j);
            const int m = min(64, y1 - c + 1);
            for (int t = 0; t < m; ++t) {
                fl += __shfl(j, t, 64);
                rs += __shfl(r, t, 64);
            }
        }
        if (lane == 0) {
            out[k] = fl;
            out[n_out + k] = rs;
        }
    } else {
        double o[5];
        boundary_ends(a.cell, a.nx, a.ny, a.pitch,
                      [&](size_t n, double &rho, double &jx) { moments(n, rho, jx); }, o);
        if (lane == 0)
#pragma unroll
            for (int q = 0; q < 5; ++q) out[2 * n_out + q] = o[q];
    }
}

// ---------------------------------------------------------------------------
// Cell word of cell (x, y) from the logical type map: wall bit of population
// i set when the pull source x - c_i is solid or off the lattice.
__device__ __forceinline__ uint32_t cell_word(const uint8_t *types, int x, int y, int nx, int ny,
                                              int flags) {
    const uint32_t t = types[(size_t)y * nx + x];
    uint32_t w = t << 8;
    if (t != kSolid) {
        const bool sym = (flags & kFlagSymmetryTop) != 0;
#pragma unroll
        for (int i = 1; i < 9; ++i) {
            // a source beyond the symmetry line is its mirror in row ny-1
            const int sx = x - kCx[i];
            int sy = y - kCy[i];
            if (sym && sy == ny) sy = ny - 1;
            const bool wall = sx < 0 || sx >= nx || sy < 0 || sy >= ny ||
                              types[(size_t)sy * nx + sx] == kSolid;
            w |= (wall ? 1u : 0u) << (i - 1);
        }
        if ((flags & kFlagNeumannOutlet) && t == kOutlet) {
            w |= kWordNeumann;
            if (x > 0 && types[(size_t)y * nx + x - 1] != kSolid) w |= kWordLeftLive;
        }
        if (sym && y == ny - 1) w |= kWordGeneral;
    }
    return w;
}

// Cell words of the whole lattice.  Pad columns are solid.
__global__ __launch_bounds__(256) void build_cells_kernel(const uint8_t *types,
                                                          uint16_t *cell,
                                                          int nx, int ny,
                                                          int pitch, int flags) {
    const int x = blockIdx.x * 64 + threadIdx.x;
    const int y = blockIdx.y * 4 + threadIdx.y;
    if (x >= pitch || y >= ny) return;
    const uint32_t w = x < nx ? cell_word(types, x, y, nx, ny, flags) : 0u;
    cell[(size_t)y * pitch + x] = (uint16_t)w;
}

// Cell words of the 3 x 3 neighbourhood of each listed cell (logical
// indices): after cells flipped, the only words that change are those of the
// flipped cells and of their eight neighbours (a cell's word depends on its
// own type and those of its eight neighbours).  Nine threads per listed cell;
// a word reached from two listed cells is written twice with the same value.
__global__ __launch_bounds__(256) void build_cells_at_kernel(const uint8_t *types, uint16_t *cell,
                                                             const int32_t *cells, int count,
                                                             int nx, int ny, int pitch,
                                                             int flags) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 9 * count) return;
    const int l = cells[t / 9], j = t % 9;
    const int x = l % nx + (j % 3) - 1, y = l / nx + (j / 3) - 1;
    if (x < 0 || x >= nx || y < 0 || y >= ny) return;
    cell[(size_t)y * pitch + x] = (uint16_t)cell_word(types, x, y, nx, ny, flags);
}

// Every population offset of the given cells to zero: the rest equilibrium
// f_i = w_i.
template <typename T>
__global__ void zero_cells_kernel(T *f, size_t plane, const int32_t *cells,
                                  int count, int nx, int pitch) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= count) return;
    const int l = cells[k];
    const size_t n = (size_t)(l / nx) * pitch + (l % nx);
#pragma unroll
    for (int i = 0; i < 9; ++i) f[(size_t)i * plane + n] = Sto<T>::from_d(0.0);
}

template <typename T>
__global__ void fill_kernel(T *p, size_t count, T v) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (size_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// State export / import of one population plane: f = w_i + d (0 on solid
// cells) in logical layout.
template <typename T>
__global__ __launch_bounds__(256) void export_plane_kernel(
    const T *f, const uint16_t *cell, double *out, int i, int nx, int ny,
    int pitch, size_t plane) {
    const int x = blockIdx.x * 64 + threadIdx.x;
    const int y = blockIdx.y * 4 + threadIdx.y;
    if (x >= nx || y >= ny) return;
    const size_t n = (size_t)y * pitch + x;
    const bool solid = cell_type(cell[n]) == kSolid;
    out[(size_t)y * nx + x] =
        solid ? 0.0 : wgt<double>(i) + Sto<T>::to_d(f[(size_t)i * plane + n]);
}

template <typename T>
__global__ __launch_bounds__(256) void import_plane_kernel(
    T *f, const uint16_t *cell, const double *in, int i, int nx, int ny,
    int pitch, size_t plane) {
    const int x = blockIdx.x * 64 + threadIdx.x;
    const int y = blockIdx.y * 4 + threadIdx.y;
    if (x >= nx || y >= ny) return;
    const size_t n = (size_t)y * pitch + x;
    const bool solid = cell_type(cell[n]) == kSolid;
    f[(size_t)i * plane + n] =
        Sto<T>::from_d(solid ? 0.0 : in[(size_t)y * nx + x] - wgt<double>(i));
}

// ---------------------------------------------------------------------------
// Exchange step (Sec. 2.2): the keys and flip kernels live in lbm_keys.h; the
// state digest below uses the same SplitMix64.
using keys::splitmix64;

// ---------------------------------------------------------------------------
// Host-side launchers.
static inline dim3 grid_cells(int ncols, int ny) {
    return dim3((unsigned)((ncols + 63) / 64), (unsigned)((ny + 3) / 4));
}

#define LBM_OFFSET_LAUNCHERS(T, CELL)                                                  \
    template <>                                                                          \
    hipError_t launch_sweep<T>(const SweepArgs<T> &a, bool check, hipStream_t s) {       \
        return sweep::launch_step<CELL>(a, check, s);                                    \
    }                                                                                    \
    template <>                                                                          \
    hipError_t launch_tb<T>(const SweepArgs<T> &a, const int32_t *tiles, int n_tiles,    \
                            int steps, bool check, int variant, hipStream_t s) {         \
        return sweep::launch_tb_variant<CELL>(a, tiles, n_tiles, steps, check, variant,  \
                                              s);                                        \
    }                                                                                    \
    template <>                                                                          \
    hipError_t launch_tb_batch<T>(const SweepArgs<T> *args, const int32_t *lat,          \
                                  const int32_t *tiles, int n_items, int steps,          \
                                  int variant, bool bc, hipStream_t s) {                 \
        return sweep::launch_tb_batch_variant<CELL>(args, lat, tiles, n_items, steps,    \
                                                    variant, bc, s);                     \
    }                                                                                    \
    template <>                                                                          \
    hipError_t launch_step_batch<T>(const SweepArgs<T> *args, const int32_t *lat,        \
                                    const int32_t *blocks, int n_items, bool bc,         \
                                    hipStream_t s) {                                     \
        return sweep::launch_step_batch<CELL>(args, lat, blocks, n_items, bc, s);        \
    }
LBM_OFFSET_LAUNCHERS(float, F32Cell)
LBM_OFFSET_LAUNCHERS(h16, H16Cell)
LBM_OFFSET_LAUNCHERS(bf16, BF16Cell)

int64_t sweep_blocks(int nx, int ny) {
    const dim3 g = grid_cells(nx, ny);
    return (int64_t)g.x * g.y;
}

hipError_t launch_finalize_check(const double *partials, int64_t count, RunControl *ctl, int j,
                                 double tol, hipStream_t s) {
    hipLaunchKernelGGL(finalize_check_kernel, dim3(1), dim3(256), 0, s, partials, count, ctl, j,
                       tol);
    return hipGetLastError();
}

hipError_t launch_finalize1(const double *partials, int64_t count, double *out,
                            hipStream_t s) {
    hipLaunchKernelGGL(finalize_kernel<1>, dim3(1), dim3(256), 0, s, partials,
                       count, out);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_macro(const MacroArgs<T> &a, hipStream_t s) {
    hipLaunchKernelGGL(macro_kernel<T>, grid_cells(a.nx, a.ny), dim3(64, 4), 0,
                       s, a);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_mass(const MacroArgs<T> &a, double *partials, hipStream_t s) {
    hipLaunchKernelGGL(mass_kernel<T>, grid_cells(a.nx, a.ny), dim3(64, 4), 0,
                       s, a, partials);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_boundary(const MacroArgs<T> &a, const int32_t *y0,
                           const int32_t *y1, int n_out, double *out,
                           hipStream_t s) {
    hipLaunchKernelGGL(boundary_kernel<T>, dim3((unsigned)(n_out + 1)), dim3(kBoundaryThreads),
                       0, s, a, y0, y1, n_out, out);
    return hipGetLastError();
}

hipError_t launch_build_cells(const uint8_t *types, uint16_t *cell, int nx,
                              int ny, int pitch, int flags, hipStream_t s) {
    hipLaunchKernelGGL(build_cells_kernel, grid_cells(pitch, ny), dim3(64, 4),
                       0, s, types, cell, nx, ny, pitch, flags);
    return hipGetLastError();
}

hipError_t launch_build_cells_at(const uint8_t *types, uint16_t *cell, const int32_t *cells,
                                 int count, int nx, int ny, int pitch, int flags,
                                 hipStream_t s) {
    if (count <= 0) return hipSuccess;
    const int64_t threads = 9 * (int64_t)count;
    hipLaunchKernelGGL(build_cells_at_kernel, dim3((unsigned)((threads + 255) / 256)), dim3(256),
                       0, s, types, cell, cells, count, nx, ny, pitch, flags);
    return hipGetLastError();
}

template <typename T>
hipError_t rest_cells_impl(T *f, size_t plane, const int32_t *cells, int count, int nx,
                           int pitch, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(zero_cells_kernel<T>, dim3((count + 255) / 256), dim3(256), 0, s, f,
                       plane, cells, count, nx, pitch);
    return hipGetLastError();
}

template <typename T>
hipError_t rest_all_impl(T *f, size_t plane, hipStream_t s) {
    const size_t count = 9 * plane;
    size_t blocks = (count + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    T zero;
    std::memset(&zero, 0, sizeof zero);  // +0 in every storage format
    hipLaunchKernelGGL(fill_kernel<T>, dim3((unsigned)blocks), dim3(256), 0, s, f, count, zero);
    return hipGetLastError();
}

#define LBM_OFFSET_REST(T)                                                             \
    template <>                                                                        \
    hipError_t launch_rest_cells<T>(T * f, size_t plane, const int32_t *cells,         \
                                    int count, int nx, int pitch, hipStream_t s) {     \
        return rest_cells_impl<T>(f, plane, cells, count, nx, pitch, s);               \
    }                                                                                  \
    template <>                                                                        \
    hipError_t launch_rest_all<T>(T * f, size_t plane, hipStream_t s) {                \
        return rest_all_impl<T>(f, plane, s);                                          \
    }
LBM_OFFSET_REST(float)
LBM_OFFSET_REST(h16)
LBM_OFFSET_REST(bf16)

template <typename T>
hipError_t launch_export_plane(const T *f, const uint16_t *cell, double *out,
                               int i, int nx, int ny, int pitch, size_t plane,
                               hipStream_t s) {
    hipLaunchKernelGGL(export_plane_kernel<T>, grid_cells(nx, ny), dim3(64, 4),
                       0, s, f, cell, out, i, nx, ny, pitch, plane);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_import_plane(T *f, const uint16_t *cell, const double *in,
                               int i, int nx, int ny, int pitch, size_t plane,
                               hipStream_t s) {
    hipLaunchKernelGGL(import_plane_kernel<T>, grid_cells(nx, ny), dim3(64, 4),
                       0, s, f, cell, in, i, nx, ny, pitch, plane);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_keys(const KeysArgs &a, hipStream_t s) {
    return keys::launch_keys<OffsetMoments<T>>(a, s);
}

template <typename T>
hipError_t launch_flip(const FlipArgs &a, hipStream_t s) {
    return keys::launch_flip<OffsetMoments<T>>(a, s);
}

// ---------------------------------------------------------------------------
// State digest: sum mod 2^64 over cells of SplitMix64 of each stored
// population's bits mixed with its logical position, plus each cell's type.
template <typename T>
__device__ __forceinline__ uint64_t raw_bits(T v) {
    uint64_t r = 0;
    __builtin_memcpy(&r, &v, sizeof(T));
    return r;
}

template <typename T>
__global__ __launch_bounds__(256) void digest_kernel(const T *f, const uint16_t *cell,
                                                     const uint8_t *types, int nx, int ny,
                                                     int pitch, size_t plane,
                                                     unsigned long long *out) {
    // Grid-stride over logical cells; one atomic per workgroup.
    __shared__ uint64_t part[4];
    const uint64_t N = (uint64_t)nx * (uint64_t)ny;
    uint64_t acc = 0;
    for (uint64_t l = (uint64_t)blockIdx.x * 256 + threadIdx.x; l < N;
         l += (uint64_t)gridDim.x * 256) {
        const int y = (int)(l / (uint64_t)nx), x = (int)(l % (uint64_t)nx);
        const size_t n = (size_t)y * pitch + x;
        acc += splitmix64((uint64_t)types[l] ^ (l << 8) ^ 0xd1b54a32d192ed03ull);
        if (cell_type(cell[n]) != kSolid) {
#pragma unroll
            for (int i = 0; i < 9; ++i)
                acc += splitmix64(raw_bits(f[(size_t)i * plane + n]) ^
                                  ((9 * l + (uint64_t)i) * 0x9e3779b97f4a7c15ull));
        }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        const uint64_t t = part[0] + part[1] + part[2] + part[3];
        if (t != 0) atomicAdd(out, (unsigned long long)t);
    }
}

template <typename T>
hipError_t launch_digest(const T *f, const uint16_t *cell, const uint8_t *types, int nx,
                         int ny, int pitch, size_t plane, unsigned long long *out,
                         hipStream_t s) {
    const uint64_t N = (uint64_t)nx * (uint64_t)ny;
    const unsigned blocks = (unsigned)std::min<uint64_t>(2048, (N + 255) / 256);
    hipLaunchKernelGGL(digest_kernel<T>, dim3(blocks), dim3(256), 0, s, f, cell, types, nx, ny,
                       pitch, plane, out);
    return hipGetLastError();
}
template hipError_t launch_digest<double>(const double *, const uint16_t *, const uint8_t *,
                                          int, int, int, size_t, unsigned long long *,
                                          hipStream_t);
template hipError_t launch_digest<float>(const float *, const uint16_t *, const uint8_t *,
                                         int, int, int, size_t, unsigned long long *,
                                         hipStream_t);
template hipError_t launch_digest<h16>(const h16 *, const uint16_t *, const uint8_t *, int,
                                       int, int, size_t, unsigned long long *, hipStream_t);
template hipError_t launch_digest<bf16>(const bf16 *, const uint16_t *, const uint8_t *, int,
                                        int, int, size_t, unsigned long long *, hipStream_t);

// Offset-storage instantiations (double precision: lbm_f64.hip).
#define LBM_OFFSET_INST(T)                                                                  \
    template hipError_t launch_macro<T>(const MacroArgs<T> &, hipStream_t);                  \
    template hipError_t launch_mass<T>(const MacroArgs<T> &, double *, hipStream_t);         \
    template hipError_t launch_boundary<T>(const MacroArgs<T> &, const int32_t *,            \
                                           const int32_t *, int, double *, hipStream_t);     \
    template hipError_t launch_export_plane<T>(const T *, const uint16_t *, double *, int,   \
                                               int, int, int, size_t, hipStream_t);          \
    template hipError_t launch_import_plane<T>(T *, const uint16_t *, const double *, int,   \
                                               int, int, int, size_t, hipStream_t);          \
    template hipError_t launch_keys<T>(const KeysArgs &, hipStream_t);                       \
    template hipError_t launch_flip<T>(const FlipArgs &, hipStream_t);
LBM_OFFSET_INST(float)
LBM_OFFSET_INST(h16)
LBM_OFFSET_INST(bf16)

}  // namespace lbm
