// Internal declarations shared by the kernels and the host library.
#pragma once

#include <hip/hip_bf16.h>
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <type_traits>

namespace lbm {

enum : uint32_t { kSolid = 0, kFluid = 1, kInlet = 2, kOutlet = 3 };
enum : int { kCritPaper = 0, kCritSpeed = 1 };

// 16-bit storage types of the reduced-precision forms.
using h16 = _Float16;
using bf16 = __hip_bfloat16;

// Conversions between a storage type and double / float (round to nearest
// even where the target is narrower).
template <typename T>
struct Sto;
template <>
struct Sto<double> {
    __device__ static __forceinline__ double to_d(double v) { return v; }
    __device__ static __forceinline__ double from_d(double v) { return v; }
};
template <>
struct Sto<float> {
    __device__ static __forceinline__ double to_d(float v) { return (double)v; }
    __device__ static __forceinline__ float from_d(double v) { return (float)v; }
    __device__ static __forceinline__ float to_f(float v) { return v; }
    __device__ static __forceinline__ float from_f(float v) { return v; }
};
// float -> IEEE binary16 with the hardware conversion (round to nearest
// even).  The empty register-only asm statement makes the float value opaque,
// so the compiler cannot fold the conversion into a preceding multiply-add
// (a fused multiply-add rounding once, directly to half): every kernel then
// rounds to float first and to half second, and stores the same bits.
__device__ __forceinline__ h16 f32_to_h16_rne(float f) {
    asm volatile("" : "+v"(f));
    return (h16)f;
}

template <>
struct Sto<h16> {
    __device__ static __forceinline__ double to_d(h16 v) { return (double)(float)v; }
    __device__ static __forceinline__ h16 from_d(double v) { return f32_to_h16_rne((float)v); }
    __device__ static __forceinline__ float to_f(h16 v) { return (float)v; }
    __device__ static __forceinline__ h16 from_f(float v) { return f32_to_h16_rne(v); }
};
template <>
struct Sto<bf16> {
    __device__ static __forceinline__ double to_d(bf16 v) { return (double)__bfloat162float(v); }
    __device__ static __forceinline__ bf16 from_d(double v) { return __float2bfloat16((float)v); }
    __device__ static __forceinline__ float to_f(bf16 v) { return __bfloat162float(v); }
    __device__ static __forceinline__ bf16 from_f(float v) { return __float2bfloat16(v); }
};

// Arguments of one sweep launch.  Populations live in nine planes of `plane`
// elements (ny rows of `pitch`).  Single precision stores the offsets
// d_i = f_i - w_i; double precision stores f_i (see lbm_f64.hip).
// Inlet velocities are double for the double form and float for the offset
// forms (never 16-bit: the imposed velocity keeps its precision).
template <typename T>
using UinT = typename std::conditional<std::is_same<T, double>::value, double, float>::type;

template <typename T>
struct SweepArgs {
    const T *fin;
    T *fout;
    const uint16_t *cell;
    const UinT<T> *uin;  // inlet velocity per row
    double *uprev;     // two planes (u_x, u_y); check steps only
    double *partials;  // 4 doubles per block; check steps only
    int nx, ny, pitch;
    size_t plane;
    double omega;      // 1 / tau
    double rho_out;
    double one_minus_rho_out;
};

template <typename T>
struct MacroArgs {
    const T *f;
    const uint16_t *cell;
    double *rho, *ux, *uy;  // logical layout, optional
    double *uprev;          // pitched, optional
    int nx, ny, pitch;
    size_t plane;
};

struct KeysArgs {
    const uint8_t *types;  // logical layout
    const double *rho, *ux, *uy;
    int nx, ny, band_x, band_y, criterion;
    uint64_t seed;
    int64_t cap;
    unsigned long long *count_f, *count_s;
    int *error;
    uint64_t *kf, *hf, *ks, *hs;
    int32_t *if_, *is;
};

template <typename T>
hipError_t launch_sweep(const SweepArgs<T> &a, bool check, hipStream_t s);

// Temporal blocking: regions of 64 x rows cells with a halo of `halo` cells
// (so up to `halo` steps per launch), tiles of (64 - 2 halo) x (rows - 2 halo)
// cells, `threads` threads per workgroup, two LDS copies of the region
// (9 * 64 * rows * sizeof(T) bytes each).
template <typename T>
struct TbShape;
#ifndef LBM_TB32_ROWS
#define LBM_TB32_ROWS 32
#endif
#ifndef LBM_TB32_HALO
#define LBM_TB32_HALO 8
#endif
#ifndef LBM_TB64_ROWS
#define LBM_TB64_ROWS 16
#endif
#ifndef LBM_TB64_HALO
#define LBM_TB64_HALO 4
#endif
template <>
struct TbShape<float> {
    static constexpr int rows = LBM_TB32_ROWS, halo = LBM_TB32_HALO, threads = 1024;
};
template <>
struct TbShape<double> {
    static constexpr int rows = LBM_TB64_ROWS, halo = LBM_TB64_HALO, threads = 1024;
};
template <>
struct TbShape<h16> {
    static constexpr int rows = 32, halo = 8, threads = 1024;
};
template <>
struct TbShape<bf16> {
    static constexpr int rows = 32, halo = 8, threads = 1024;
};
template <typename T>
constexpr int tile_w() { return 64 - 2 * TbShape<T>::halo; }
template <typename T>
constexpr int tile_h() { return TbShape<T>::rows - 2 * TbShape<T>::halo; }
// `steps` (1..TbShape<T>::halo) time steps on the listed tiles; with `check` the last
// step also writes per-tile residual partials (4 doubles per tile).
template <typename T>
hipError_t launch_tb(const SweepArgs<T> &a, const int32_t *tiles, int n_tiles, int steps,
                     bool check, hipStream_t s);
int64_t sweep_blocks(int nx, int ny);
hipError_t launch_finalize4(const double *partials, int64_t count, double *out,
                            hipStream_t s);
hipError_t launch_finalize1(const double *partials, int64_t count, double *out,
                            hipStream_t s);
template <typename T>
hipError_t launch_macro(const MacroArgs<T> &a, hipStream_t s);
template <typename T>
hipError_t launch_mass(const MacroArgs<T> &a, double *partials, hipStream_t s);
template <typename T>
hipError_t launch_boundary(const MacroArgs<T> &a, const int32_t *y0,
                           const int32_t *y1, int n_out, double *out,
                           hipStream_t s);
hipError_t launch_build_cells(const uint8_t *types, uint16_t *cell, int nx,
                              int ny, int pitch, hipStream_t s);
// Put the given cells (logical indices) / the whole buffer at rest
// (f_i = w_i: offsets 0 in single precision, w_i in double precision).
template <typename T>
hipError_t launch_rest_cells(T *f, size_t plane, const int32_t *cells,
                             int count, int nx, int pitch, hipStream_t s);
template <typename T>
hipError_t launch_rest_all(T *f, size_t plane, hipStream_t s);
template <typename T>
hipError_t launch_export_plane(const T *f, const uint16_t *cell, double *out,
                               int i, int nx, int ny, int pitch, size_t plane,
                               hipStream_t s);
template <typename T>
hipError_t launch_import_plane(T *f, const uint16_t *cell, const double *in,
                               int i, int nx, int ny, int pitch, size_t plane,
                               hipStream_t s);
hipError_t launch_keys(const KeysArgs &a, hipStream_t s);
hipError_t launch_rank(const uint64_t *key, const uint64_t *hash,
                       const int32_t *idx, int64_t count, int64_t k_eff,
                       int32_t *sel, hipStream_t s);
hipError_t launch_flip(uint8_t *types, const int32_t *removed,
                       const int32_t *added, int k_eff, double *mass_out,
                       const double *rho, hipStream_t s);
hipError_t launch_count_type(const uint8_t *types, size_t count, uint8_t which,
                             unsigned long long *out, hipStream_t s);

// Double-precision specialisations, defined in lbm_f64.hip.
template <>
hipError_t launch_sweep<double>(const SweepArgs<double> &a, bool check, hipStream_t s);
template <>
hipError_t launch_tb<double>(const SweepArgs<double> &a, const int32_t *tiles, int n_tiles,
                             int steps, bool check, hipStream_t s);
template <>
hipError_t launch_macro<double>(const MacroArgs<double> &a, hipStream_t s);
template <>
hipError_t launch_mass<double>(const MacroArgs<double> &a, double *partials, hipStream_t s);
template <>
hipError_t launch_boundary<double>(const MacroArgs<double> &a, const int32_t *y0,
                                   const int32_t *y1, int n_out, double *out, hipStream_t s);
template <>
hipError_t launch_rest_cells<double>(double *f, size_t plane, const int32_t *cells,
                                     int count, int nx, int pitch, hipStream_t s);
template <>
hipError_t launch_rest_all<double>(double *f, size_t plane, hipStream_t s);
template <>
hipError_t launch_export_plane<double>(const double *f, const uint16_t *cell, double *out,
                                       int i, int nx, int ny, int pitch, size_t plane,
                                       hipStream_t s);
template <>
hipError_t launch_import_plane<double>(double *f, const uint16_t *cell, const double *in,
                                       int i, int nx, int ny, int pitch, size_t plane,
                                       hipStream_t s);
// Single- and half-precision storage specialisations, defined in
// lbm_kernels.hip.
#define LBM_DECLARE_OFFSET(T)                                                             \
    template <>                                                                            \
    hipError_t launch_sweep<T>(const SweepArgs<T> &a, bool check, hipStream_t s);          \
    template <>                                                                            \
    hipError_t launch_tb<T>(const SweepArgs<T> &a, const int32_t *tiles, int n_tiles,      \
                            int steps, bool check, hipStream_t s);                         \
    template <>                                                                            \
    hipError_t launch_rest_cells<T>(T * f, size_t plane, const int32_t *cells, int count,  \
                                    int nx, int pitch, hipStream_t s);                     \
    template <>                                                                            \
    hipError_t launch_rest_all<T>(T * f, size_t plane, hipStream_t s);
LBM_DECLARE_OFFSET(float)
LBM_DECLARE_OFFSET(h16)
LBM_DECLARE_OFFSET(bf16)

}  // namespace lbm
