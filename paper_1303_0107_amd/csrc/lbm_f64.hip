// Double-precision kernels of the D2Q9 sweep, in the reference arithmetic
// form: populations stored as full f_i (post-collision), and every
// floating-point expression evaluated in the order the method's definition
// writes it (moments summed in population order, equilibrium of Sec. 2.1
// expanded as written, relaxation f - (1/tau)(f - feq) of Eq. 1, Zou-He
// closures as printed).  This file is compiled with -ffp-contract=off, so no
// multiply-add is fused and each operation rounds once, as IEEE-754 double
// arithmetic on any conforming machine does: results are reproducible bit
// for bit.  Wang, Fan & Luo, Sec. 2.1 (Eqs. 1-2), Sec. 3.3 (boundaries),
// Sec. 4.2 (Eqs. 9-11), Eq. 4.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lbm_boundary.h"
#include "lbm_internal.h"
#include "lbm_keys.h"

#pragma clang fp contract(off)

#include "lbm_sweep.h"

namespace lbm {
namespace f64 {

__device__ constexpr int kCx[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
__device__ constexpr int kCy[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
__device__ constexpr int kOpp[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};

__device__ __forceinline__ double weight(int i) {
    return i == 0 ? 4.0 / 9.0 : (i < 5 ? 1.0 / 9.0 : 1.0 / 36.0);
}

// rho = sum f_i, j = sum c_i f_i (Eq. 2), each summed in population order.
__device__ __forceinline__ void moments(const double (&f)[9], double &r,
                                        double &mx, double &my) {
    r = 0.0;
    mx = 0.0;
    my = 0.0;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        r += f[i];
        mx += kCx[i] * f[i];
        my += kCy[i] * f[i];
    }
}

// Density and velocity of cell n (pitched) of the stored state: the
// macroscopic export and the exchange-step keys both use this.
struct Moments {
    using T = double;
    __device__ static __forceinline__ void at(const double *f, size_t plane, size_t n,
                                              double &r, double &ux, double &uy) {
        double g[9], mx, my;
#pragma unroll
        for (int i = 0; i < 9; ++i) g[i] = f[(size_t)i * plane + n];
        moments(g, r, mx, my);
        ux = mx / r;
        uy = my / r;
    }
};

template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], int tid) {
    __shared__ double red[4][NV];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
#pragma unroll
        for (int k = 0; k < NV; ++k) v[k] += __shfl_xor(v[k], off, 64);
    if ((tid & 63) == 0)
#pragma unroll
        for (int k = 0; k < NV; ++k) red[tid >> 6][k] = v[k];
    __syncthreads();
    if (tid == 0)
#pragma unroll
        for (int k = 0; k < NV; ++k) v[k] = ((red[0][k] + red[1][k]) + red[2][k]) + red[3][k];
}

// One cell of one time step on full populations: Zou-He closure on inlet
// (velocity u_in, unknowns 1, 5, 8) and outlet cells (density rho_out, zero
// transverse velocity, unknowns 3, 6, 7), moments (Eq. 2), relaxation
// f - (1/tau)(f - feq) (Eq. 1) to the equilibrium of Sec. 2.1.
struct Cell {
    using T = double;
    using CT = ArithT<double>;
    __device__ static __forceinline__ double load(double v) { return v; }
    __device__ static __forceinline__ double store(double v) { return v; }
    // Velocity (Eq. 2) of a stored population set, formed as the oracle does.
    __device__ static __forceinline__ void velocity(double (&g)[9], double &ux, double &uy) {
        double r, mx, my;
        moments(g, r, mx, my);
        ux = mx / r;
        uy = my / r;
    }
    // (bx, by): the inlet velocity (inlet cells) or the velocity a Neumann
    // outlet imposes (that of its x-1 neighbour's stored state).
    __device__ static __forceinline__ void update(double (&f)[9], uint32_t type, double bx,
                                                  double by, const SweepArgs<double> &a,
                                                  double &mass, double &ux, double &uy) {
        if (type == kInlet) {
            const double rho = (f[0] + f[2] + f[4] + 2.0 * (f[3] + f[6] + f[7])) / (1.0 - bx);
            const double ru = rho * bx;
            f[1] = f[3] + (2.0 / 3.0) * ru;
            f[5] = f[7] - 0.5 * (f[2] - f[4]) + (1.0 / 6.0) * ru;
            f[8] = f[6] + 0.5 * (f[2] - f[4]) + (1.0 / 6.0) * ru;
        } else if (type == kOutlet) {
            const double uo =
                -1.0 + (f[0] + f[2] + f[4] + 2.0 * (f[1] + f[5] + f[8])) / a.rho_out;
            const double ru = a.rho_out * uo;
            f[3] = f[1] - (2.0 / 3.0) * ru;
            f[7] = f[5] + 0.5 * (f[2] - f[4]) - (1.0 / 6.0) * ru;
            f[6] = f[8] - 0.5 * (f[2] - f[4]) - (1.0 / 6.0) * ru;
        } else if (type == kOutletNeumann) {
            const double rho = (f[0] + f[2] + f[4] + 2.0 * (f[1] + f[5] + f[8])) / (1.0 + bx);
            const double ru = rho * bx, rv = rho * by;
            f[3] = f[1] - (2.0 / 3.0) * ru;
            f[7] = f[5] + 0.5 * (f[2] - f[4]) - (1.0 / 6.0) * ru - 0.5 * rv;
            f[6] = f[8] - 0.5 * (f[2] - f[4]) - (1.0 / 6.0) * ru + 0.5 * rv;
        }
        double r, mx, my;
        moments(f, r, mx, my);
        ux = mx / r;
        uy = my / r;
        const double uu = ux * ux + uy * uy;
        const double om = a.omega;
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            const double cu = kCx[i] * ux + kCy[i] * uy;
            const double feq =
                weight(i) * r * (1.0 + cu * 3.0 + 0.5 * (cu * cu) * 9.0 - 0.5 * uu * 3.0);
            f[i] = f[i] - om * (f[i] - feq);
        }
        mass = r;
    }
};

__global__ __launch_bounds__(256) void macro_kernel(MacroArgs<double> a) {
    const int x = blockIdx.x * 64 + threadIdx.x;
    const int y = blockIdx.y * 4 + threadIdx.y;
    if (x >= a.nx || y >= a.ny) return;
    const size_t n = (size_t)y * a.pitch + x;
    const size_t l = (size_t)y * a.nx + x;
    double r = 0.0, ux = 0.0, uy = 0.0;
    if (cell_type(a.cell[n]) != kSolid) Moments::at(a.f, a.plane, n, r, ux, uy);
    if (a.rho) {
        a.rho[l] = r;
        a.ux[l] = ux;
        a.uy[l] = uy;
    }
    if (a.uprev) {
        a.uprev[n] = ux;
        a.uprev[a.plane + n] = uy;
    }
}

__global__ __launch_bounds__(256) void mass_kernel(MacroArgs<double> a,
                                                   double *partials) {
    const int x = blockIdx.x * 64 + threadIdx.x;
    const int y = blockIdx.y * 4 + threadIdx.y;
    double v[1] = {0.0};
    if (x < a.nx && y < a.ny) {
        const size_t n = (size_t)y * a.pitch + x;
        if (cell_type(a.cell[n]) != kSolid) {
            double f[9], mx, my;
#pragma unroll
            for (int i = 0; i < 9; ++i) f[i] = a.f[(size_t)i * a.plane + n];
            moments(f, v[0], mx, my);
        }
    }
    const int tid = threadIdx.y * 64 + threadIdx.x;
    block_sum<1>(v, tid);
    if (tid == 0) partials[(size_t)blockIdx.y * gridDim.x + blockIdx.x] = v[0];
}

// Boundary sums in increasing y: workgroup k < n_out sums the x momentum of
// outlet k; workgroup n_out sums x momentum and density over the inlet cells
// and density over all outlet cells (one running sum each).  out layout:
// [flow_0..flow_{n-1}, unused n, flow_in, rho_in, count_in, count_out, rho_out]
__global__ __launch_bounds__(kBoundaryThreads) void boundary_kernel(MacroArgs<double> a,
                                                                    const int32_t *out_y0,
                                                                    const int32_t *out_y1,
                                                                    int n_out, double *out) {
    // The sums take the rows in increasing y one at a time (the oracle's
    // sequential order): an outlet's rows are read by one wave, 64 at once,
    // the inlet and all outlet cells by the whole workgroup (boundary_ends).
    const int k = blockIdx.x, lane = threadIdx.x;
    auto at = [&](size_t n, double &r, double &mx) {
        double f[9], my;
#pragma unroll
        for (int i = 0; i < 9; ++i) f[i] = a.f[(size_t)i * a.plane + n];
        moments(f, r, mx, my);
    };
    if (k < n_out) {
        if (threadIdx.x >= 64) return;  // one wave per outlet
        const int y0 = out_y0[k], y1 = out_y1[k];
        double fl = 0.0;
        for (int c = y0; c <= y1; c += 64) {
            double r = 0.0, mx = 0.0;
            if (c + lane <= y1) at((size_t)(c + lane) * a.pitch + (a.nx - 1), r, mx);
            const int m = min(64, y1 - c + 1);
            for (int t = 0; t < m; ++t) fl += __shfl(mx, t, 64);
        }
        if (lane == 0) {
            out[k] = fl;
            out[n_out + k] = 0.0;
        }
    } else {
        double o[5];
        boundary_ends(a.cell, a.nx, a.ny, a.pitch,
                      [&](size_t n, double &r, double &mx) { at(n, r, mx); }, o);
        if (lane == 0)
#pragma unroll
            for (int q = 0; q < 5; ++q) out[2 * n_out + q] = o[q];
    }
}

__global__ void rest_cells_kernel(double *f, size_t plane, const int32_t *cells,
                                  int count, int nx, int pitch) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= count) return;
    const int l = cells[k];
    const size_t n = (size_t)(l / nx) * pitch + (l % nx);
#pragma unroll
    for (int i = 0; i < 9; ++i) f[(size_t)i * plane + n] = weight(i);
}

__global__ void rest_all_kernel(double *f, size_t plane) {
    for (size_t j = (size_t)blockIdx.x * blockDim.x + threadIdx.x; j < plane;
         j += (size_t)gridDim.x * blockDim.x)
#pragma unroll
        for (int i = 0; i < 9; ++i) f[(size_t)i * plane + j] = weight(i);
}

__global__ __launch_bounds__(256) void export_plane_kernel(
    const double *f, const uint16_t *cell, double *out, int i, int nx, int ny,
    int pitch, size_t plane) {
    const int x = blockIdx.x * 64 + threadIdx.x;
    const int y = blockIdx.y * 4 + threadIdx.y;
    if (x >= nx || y >= ny) return;
    const size_t n = (size_t)y * pitch + x;
    out[(size_t)y * nx + x] = cell_type(cell[n]) == kSolid ? 0.0 : f[(size_t)i * plane + n];
}

__global__ __launch_bounds__(256) void import_plane_kernel(
    double *f, const uint16_t *cell, const double *in, int i, int nx, int ny,
    int pitch, size_t plane) {
    const int x = blockIdx.x * 64 + threadIdx.x;
    const int y = blockIdx.y * 4 + threadIdx.y;
    if (x >= nx || y >= ny) return;
    const size_t n = (size_t)y * pitch + x;
    f[(size_t)i * plane + n] = cell_type(cell[n]) == kSolid ? weight(i) : in[(size_t)y * nx + x];
}

}  // namespace f64

static inline dim3 grid_cells(int ncols, int ny) {
    return dim3((unsigned)((ncols + 63) / 64), (unsigned)((ny + 3) / 4));
}

template <>
hipError_t launch_sweep<double>(const SweepArgs<double> &a, bool check, hipStream_t s) {
    return sweep::launch_step<f64::Cell>(a, check, s);
}

template <>
hipError_t launch_tb<double>(const SweepArgs<double> &a, const int32_t *tiles, int n_tiles,
                             int steps, bool check, int variant, hipStream_t s) {
    return sweep::launch_tb_variant<f64::Cell>(a, tiles, n_tiles, steps, check, variant, s);
}

template <>
hipError_t launch_tb_batch<double>(const SweepArgs<double> *args, const int32_t *lat,
                                   const int32_t *tiles, int n_items, int steps, int variant,
                                   bool bc, hipStream_t s) {
    return sweep::launch_tb_batch_variant<f64::Cell>(args, lat, tiles, n_items, steps, variant,
                                                     bc, s);
}

template <>
hipError_t launch_step_batch<double>(const SweepArgs<double> *args, const int32_t *lat,
                                     const int32_t *blocks, int n_items, bool bc,
                                     hipStream_t s) {
    return sweep::launch_step_batch<f64::Cell>(args, lat, blocks, n_items, bc, s);
}

template <>
hipError_t launch_macro<double>(const MacroArgs<double> &a, hipStream_t s) {
    hipLaunchKernelGGL(f64::macro_kernel, grid_cells(a.nx, a.ny), dim3(64, 4), 0, s, a);
    return hipGetLastError();
}

template <>
hipError_t launch_keys<double>(const KeysArgs &a, hipStream_t s) {
    return keys::launch_keys<f64::Moments>(a, s);
}

template <>
hipError_t launch_flip<double>(const FlipArgs &a, hipStream_t s) {
    return keys::launch_flip<f64::Moments>(a, s);
}

template <>
hipError_t launch_mass<double>(const MacroArgs<double> &a, double *partials,
                               hipStream_t s) {
    hipLaunchKernelGGL(f64::mass_kernel, grid_cells(a.nx, a.ny), dim3(64, 4), 0, s, a,
                       partials);
    return hipGetLastError();
}

template <>
hipError_t launch_boundary<double>(const MacroArgs<double> &a, const int32_t *y0,
                                   const int32_t *y1, int n_out, double *out,
                                   hipStream_t s) {
    hipLaunchKernelGGL(f64::boundary_kernel, dim3((unsigned)(n_out + 1)), dim3(kBoundaryThreads),
                       0, s, a, y0, y1, n_out, out);
    return hipGetLastError();
}

template <>
hipError_t launch_rest_cells<double>(double *f, size_t plane, const int32_t *cells,
                                     int count, int nx, int pitch, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(f64::rest_cells_kernel, dim3((count + 255) / 256), dim3(256), 0, s,
                       f, plane, cells, count, nx, pitch);
    return hipGetLastError();
}

template <>
hipError_t launch_rest_all<double>(double *f, size_t plane, hipStream_t s) {
    size_t blocks = (plane + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(f64::rest_all_kernel, dim3((unsigned)blocks), dim3(256), 0, s, f,
                       plane);
    return hipGetLastError();
}

template <>
hipError_t launch_export_plane<double>(const double *f, const uint16_t *cell, double *out,
                                       int i, int nx, int ny, int pitch, size_t plane,
                                       hipStream_t s) {
    hipLaunchKernelGGL(f64::export_plane_kernel, grid_cells(nx, ny), dim3(64, 4), 0, s, f,
                       cell, out, i, nx, ny, pitch, plane);
    return hipGetLastError();
}

template <>
hipError_t launch_import_plane<double>(double *f, const uint16_t *cell, const double *in,
                                       int i, int nx, int ny, int pitch, size_t plane,
                                       hipStream_t s) {
    hipLaunchKernelGGL(f64::import_plane_kernel, grid_cells(nx, ny), dim3(64, 4), 0, s, f,
                       cell, in, i, nx, ny, pitch, plane);
    return hipGetLastError();
}

}  // namespace lbm
