// Internal declarations shared by the kernels and the host library.
#pragma once

#include <hip/hip_bf16.h>
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <type_traits>

struct lbm_handle;

namespace lbm {

enum : uint32_t { kSolid = 0, kFluid = 1, kInlet = 2, kOutlet = 3 };
enum : int { kCritPaper = 0, kCritSpeed = 1 };
// Lattice-wide boundary variants (Sec. 3.3): a zero-gradient outlet, and a
// symmetry plane just above the top row (the lattice is a half domain).
enum : int { kFlagNeumannOutlet = 1, kFlagSymmetryTop = 2 };

// Cell words (uint16): bits 0..7 wall flags of populations 1..8, bits 8..9
// the type; bit 10: an outlet with the zero-gradient (Neumann) closure; bit
// 11: the cell's pulls need the general rule (top row under a symmetry
// plane); bit 12: the cell at x-1 is not solid (its velocity is the one a
// Neumann outlet imposes).
enum : uint32_t {
    kWordNeumann = 1u << 10,
    kWordGeneral = 1u << 11,
    kWordLeftLive = 1u << 12
};
// Type code the per-cell update sees for a Neumann outlet.
enum : uint32_t { kOutletNeumann = 4 };
__host__ __device__ __forceinline__ uint32_t cell_type(uint32_t w) { return (w >> 8) & 3u; }
__host__ __device__ __forceinline__ uint32_t update_type(uint32_t w) {
    return (w & kWordNeumann) ? kOutletNeumann : cell_type(w);
}

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

// FP16 offsets are stored scaled by 2^12: |f - w| rarely exceeds 0.2, so the
// scaled values stay far below binary16's largest finite value, and offsets
// down to 1.5e-8 keep binary16's full 11-bit precision instead of falling into
// its subnormal range (below 6.1e-5 unscaled).  Scaling by a power of two is
// exact in float, so the only rounding is binary16's.
constexpr float kH16Scale = 4096.0f, kH16Unscale = 1.0f / 4096.0f;
template <>
struct Sto<h16> {
    __device__ static __forceinline__ double to_d(h16 v) {
        return (double)((float)v * kH16Unscale);
    }
    __device__ static __forceinline__ h16 from_d(double v) {
        return f32_to_h16_rne((float)v * kH16Scale);
    }
    __device__ static __forceinline__ float to_f(h16 v) { return (float)v * kH16Unscale; }
    __device__ static __forceinline__ h16 from_f(float v) { return f32_to_h16_rne(v * kH16Scale); }
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
// Arithmetic type of the per-cell update for a storage type: double for the
// double form, float for every offset form.  The cell policies are built from
// it and lbm_precision_info reports it.
template <typename T>
using ArithT = typename std::conditional<std::is_same<T, double>::value, double, float>::type;

struct RunControl;
// Queued runs on lattices of at most this many tiles let the first launch of
// each interval carry out the finalize step of the interval before it.
constexpr int kDeferMaxPartials = 512;

template <typename T>
struct SweepArgs {
    const T *fin;
    T *fout;
    const uint16_t *cell;
    const UinT<T> *uin;  // inlet velocity per row
    double *uprev;     // two planes (u_x, u_y); check steps only
    double *partials;  // 4 doubles per block; check steps only
    // 64 copies of a flag (one per lane, so that it is read with a vector
    // load issued beside the region's loads): nonzero when the run this
    // launch belongs to has already ended on the device, and the launch then
    // changes nothing.  Read by the single-lattice blocked kernels only.
    const int *stop;
    int nx, ny, pitch;
    size_t plane;
    double omega;      // 1 / tau
    double rho_out;
    double one_minus_rho_out;
    int flags;         // kFlagNeumannOutlet | kFlagSymmetryTop
    // Set on the first launch of interval j >= 1 of a queued run when the
    // tile list holds at most kDeferMaxPartials tiles and that launch is not
    // the interval's check launch (single-lattice blocked kernels, a kernel
    // of its own): the launch first carries out the finalize step of
    // interval prev_j = j - 1 (RunControl) from that interval's prev_count
    // partials with tolerance tol, and writes the stop flag's lane copies to
    // stop_out, in place of a finalize launch.  Null otherwise.
    const double *prev = nullptr;
    int *stop_out = nullptr;
    RunControl *ctl = nullptr;
    int prev_j = 0, prev_count = 0;
    double tol = 0.0;
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

// Exchange-step keys: from the field (rho, ux, uy; logical layout) when rho
// is given, else from the stored state f (storage of the handle, pitched).
struct KeysArgs {
    const uint8_t *types;  // logical layout
    const double *rho, *ux, *uy;
    const void *f;
    size_t plane;
    int pitch;
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
// cells, 1024 threads per workgroup, two LDS copies of the region
// (9 * 64 * rows * sizeof(T) bytes each; one copy in the in-place form) and,
// in the compacted form, a list of the region's non-solid cells (4 bytes per
// region cell); at most 160 KB in all.  A few shapes are compiled per storage type; variant 0 is the
// default, the autotuner may pick another.  The shape never changes the
// results, only the speed.
// Region bodies: dense (a lane per region column), compacted (lanes take
// consecutive entries of a list of the region's non-solid cells), or dense
// with one region copy updated in place (half the LDS, so taller regions).
enum TbKind : int { kTbDense = 0, kTbCompact = 1, kTbInPlace = 2 };
struct TbVariant {
    int rows, halo, kind;
};
template <typename T>
struct TbVariants;
template <>
struct TbVariants<double> {
    static constexpr int count = 4;
    static constexpr TbVariant v[4] = {
        {16, 4, kTbCompact}, {16, 4, kTbDense}, {16, 2, kTbCompact}, {32, 8, kTbInPlace}};
};
template <>
struct TbVariants<float> {
    static constexpr int count = 6;
    static constexpr TbVariant v[6] = {{32, 8, kTbCompact}, {32, 8, kTbDense},
                                       {32, 4, kTbCompact}, {16, 4, kTbCompact},
                                       {16, 4, kTbDense},   {32, 9, kTbDense}};
};
template <>
struct TbVariants<h16> : TbVariants<float> {};
template <>
struct TbVariants<bf16> : TbVariants<float> {};
constexpr int kTbThreads = 1024;
template <typename T>
constexpr int tile_w(int variant) { return 64 - 2 * TbVariants<T>::v[variant].halo; }
template <typename T>
constexpr int tile_h(int variant) {
    return TbVariants<T>::v[variant].rows - 2 * TbVariants<T>::v[variant].halo;
}
// `steps` (1..halo) time steps on the listed tiles with region shape
// `variant`; with `check` the last step also writes per-tile residual
// partials (4 doubles per tile).
template <typename T>
hipError_t launch_tb(const SweepArgs<T> &a, const int32_t *tiles, int n_tiles, int steps,
                     bool check, int variant, hipStream_t s);
// The same for many lattices at once: item b is tile tiles[b] of lattice
// lat[b] with arguments args[lat[b]] (device arrays); no residual partials.
// bc: some member has boundary-variant flags.
template <typename T>
hipError_t launch_tb_batch(const SweepArgs<T> *args, const int32_t *lat, const int32_t *tiles,
                           int n_items, int steps, int variant, bool bc, hipStream_t s);
// One time step of many lattices: item b is the 64 x 4 block blocks[b] of
// lattice lat[b] with arguments args[lat[b]] (device arrays).
template <typename T>
hipError_t launch_step_batch(const SweepArgs<T> *args, const int32_t *lat,
                             const int32_t *blocks, int n_items, bool bc, hipStream_t s);
int64_t sweep_blocks(int nx, int ny);
// Limits of lbm_outlet_stats_noalloc (its device scratch is a fixed array).
constexpr size_t kNoAllocScratchBytes = (size_t)1 << 20;
constexpr int kNoAllocMaxOutlets = 1024;
// Device control block of a run to steady state: the run's check intervals
// are queued several at a time, and each interval's finalize step records the
// interval's sums, counts it, and ends the run (stop = 1 converged, 2
// unstable) so that the launches queued after it change nothing.
constexpr int kRunBatchMax = 64;
struct RunControl {
    double sums[kRunBatchMax][4];
    int stop;
    int done;            // intervals of the current batch carried out
    // Copies of stop, one per lane (SweepArgs::stop), in two arrays: the
    // launches of interval j read [j % 2], except those after the first
    // launch of an interval whose first launch decides the interval before
    // it (SweepArgs::prev): that launch writes the decision to [(j + 1) % 2],
    // which the rest of the interval reads, so that no launch writes an array
    // it reads.  A finalize launch writes both.
    int stop_lanes[2][64];
    int zeros[64];       // SweepArgs::stop outside a queued run
};
// Sums of interval j into ctl->sums[j] (thread t < 256 adds partials t,
// t + 256, ..., then the block adds the threads' sums in a fixed order), then
// the stop decision: unstable if sums[3] != 0 or a sum is not finite, else
// converged if tol > 0 and sqrt(num)/sqrt(den) < tol.  Does nothing once
// ctl->stop is set.
hipError_t launch_finalize_check(const double *partials, int64_t count, RunControl *ctl, int j,
                                 double tol, hipStream_t s);
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
                              int ny, int pitch, int flags, hipStream_t s);
// The cell words of the 3 x 3 neighbourhoods of `count` listed cells (logical
// indices; device array), after those cells changed type.
hipError_t launch_build_cells_at(const uint8_t *types, uint16_t *cell, const int32_t *cells,
                                 int count, int nx, int ny, int pitch, int flags,
                                 hipStream_t s);
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
// Order-free 64-bit digest of the stored state and the type map, added to *out.
template <typename T>
hipError_t launch_digest(const T *f, const uint16_t *cell, const uint8_t *types, int nx,
                         int ny, int pitch, size_t plane, unsigned long long *out,
                         hipStream_t s);
template <typename T>
hipError_t launch_keys(const KeysArgs &a, hipStream_t s);
// The k_eff first of the nf fluid and of the ns solid candidates, each list in
// the order (key, hash), written as cell indices to sel_f and sel_s.
// `scratch` holds select_scratch_bytes(k_max) bytes, k_eff <= k_max and
// k_eff <= min(nf, ns).  An inconsistency the kernels detect (impossible for
// candidates with distinct hashes) sets bits 8 and up of *error (device).
size_t select_scratch_bytes(int64_t k_max);
hipError_t launch_select_pair(const uint64_t *kf, const uint64_t *hf, const int32_t *if_,
                              int64_t nf, const uint64_t *ks, const uint64_t *hs,
                              const int32_t *is, int64_t ns, int64_t k_eff, int32_t *sel_f,
                              int32_t *sel_s, void *scratch, int64_t k_max, int *error,
                              hipStream_t s);
// Flip the selected cells; removed_rho[k] = the density of cell removed[k],
// from the field rho (logical layout) when given, else from the stored state
// f (storage T, pitched).
struct FlipArgs {
    uint8_t *types;
    const int32_t *removed, *added;
    int k_eff;
    double *removed_rho;
    const double *rho;
    const void *f;
    size_t plane;
    int nx, pitch;
};
template <typename T>
hipError_t launch_flip(const FlipArgs &a, hipStream_t s);

// Move a handle's device work to another stream (the request server makes
// handles on a stream of its own, then runs them on the worker's).  The
// caller has synchronised the handle's current stream.
void handle_set_stream(lbm_handle *h, hipStream_t s);

// Double-precision specialisations, defined in lbm_f64.hip.
template <>
hipError_t launch_sweep<double>(const SweepArgs<double> &a, bool check, hipStream_t s);
template <>
hipError_t launch_tb<double>(const SweepArgs<double> &a, const int32_t *tiles, int n_tiles,
                             int steps, bool check, int variant, hipStream_t s);
template <>
hipError_t launch_tb_batch<double>(const SweepArgs<double> *args, const int32_t *lat,
                                   const int32_t *tiles, int n_items, int steps, int variant,
                                   bool bc, hipStream_t s);
template <>
hipError_t launch_step_batch<double>(const SweepArgs<double> *args, const int32_t *lat,
                                     const int32_t *blocks, int n_items, bool bc,
                                     hipStream_t s);
template <>
hipError_t launch_macro<double>(const MacroArgs<double> &a, hipStream_t s);
template <>
hipError_t launch_keys<double>(const KeysArgs &a, hipStream_t s);
template <>
hipError_t launch_flip<double>(const FlipArgs &a, hipStream_t s);
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
                            int steps, bool check, int variant, hipStream_t s);            \
    template <>                                                                            \
    hipError_t launch_tb_batch<T>(const SweepArgs<T> *args, const int32_t *lat,            \
                                  const int32_t *tiles, int n_items, int steps,            \
                                  int variant, bool bc, hipStream_t s);                    \
    template <>                                                                            \
    hipError_t launch_step_batch<T>(const SweepArgs<T> *args, const int32_t *lat,          \
                                    const int32_t *blocks, int n_items, bool bc,           \
                                    hipStream_t s);                                        \
    template <>                                                                            \
    hipError_t launch_rest_cells<T>(T * f, size_t plane, const int32_t *cells, int count,  \
                                    int nx, int pitch, hipStream_t s);                     \
    template <>                                                                            \
    hipError_t launch_rest_all<T>(T * f, size_t plane, hipStream_t s);
LBM_DECLARE_OFFSET(float)
LBM_DECLARE_OFFSET(h16)
LBM_DECLARE_OFFSET(bf16)

}  // namespace lbm
