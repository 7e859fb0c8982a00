/*
 * lbm.h - C ABI of the MI355X (gfx950) lattice-Boltzmann shape-optimisation
 * library.
 *
 * The library implements the hot path of the method of Wang, Fan & Luo,
 * "Lattice Boltzmann method for shape optimization of fluid distributor":
 * a D2Q9 BGK lattice-Boltzmann solve over a solid/fluid cell map (Sec. 2.1),
 * the outlet flow-rate and pressure-drop reductions used to judge a shape
 * (Eq. 4, Eqs. 9-11), and the constant-volume exchange of interface cells
 * driven by the viscous-stress and dynamic-pressure criteria (Sec. 2.2,
 * Eqs. 5-6).  The calls follow the optimisation loop of Sec. 2.3:
 *   step (1)  lbm_create_geometry
 *   step (2)  lbm_run_to_steady
 *   step (3)  lbm_shape_update
 *   step (4)  lbm_shape_update (re-initialisation) + lbm_run_to_steady
 *   step (5)  lbm_outlet_stats (pressure drop, flow uniformity)
 *
 * Conventions shared by every call
 *   - Every call returns an int status: LBM_OK (0), a warning (> 0) or an
 *     error (< 0).  lbm_last_error() then returns a message for the calling
 *     thread.  No C++ exception crosses this interface.
 *   - Lattice nx x ny; cell (x, y) has the logical index n = y*nx + x
 *     (row-major, y outer).  x = 0 is the inlet side, x = nx-1 the outlet side.
 *   - Host arrays are owned by the caller and are only read or written during
 *     the call; calls that fill host arrays return after the copy completed.
 *   - A handle owns its device memory.  It is not thread-safe; distinct
 *     handles are independent.  All device work of a handle is issued on the
 *     stream given at creation (NULL: the null stream of the current device).
 *   - Population index i follows the D2Q9 numbering of Sec. 2.1:
 *     c0 = (0,0); c1..c4 = (1,0), (0,1), (-1,0), (0,-1);
 *     c5..c8 = (1,1), (-1,1), (-1,-1), (1,-1).
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define LBM_OK 0
#define LBM_NOT_CONVERGED 1 /* run ended at max_steps above tol            */
#define LBM_EINVAL (-1)     /* bad argument or cell map                    */
#define LBM_ENOMEM (-2)     /* device allocation failed                    */
#define LBM_EHIP (-3)       /* HIP runtime error                           */
#define LBM_EUNSTABLE (-4)  /* non-finite density or velocity detected     */

/* ---- cell types (Sec. 3.3, Fig. 5) ---------------------------------------
 * Inlet cells may only sit in column 0 and outlet cells in column nx-1. */
#define LBM_SOLID 0
#define LBM_FLUID 1
#define LBM_INLET 2
#define LBM_OUTLET 3

/* ---- precision forms ------------------------------------------------------
 * LBM_F64:        populations f_i stored in double, relaxed in double, in
 *                 the reference operation order (bitwise reproducible).
 * LBM_F32:        offsets f_i - w_i stored in float, relaxed in float (a
 *                 relaxation that conserves mass and momentum exactly).
 * LBM_F32_S_F16:  offsets stored in half (IEEE binary16, scaled by 2^12),
 *                 relaxed in float.
 * LBM_F32_S_BF16: offsets stored in bfloat16, relaxed in float.
 * Reductions (mass, fluxes, pressure drop, residual, exchange keys) are
 * double in every form. */
#define LBM_F64 0
#define LBM_F32 1
#define LBM_F32_S_F16 2
#define LBM_F32_S_BF16 3

/* Bytes of one stored population value and of the floating-point type the
 * per-cell update computes in, for a precision form (the two words after
 * "stored in" and "relaxed in" above).  Needs no device.
 * Errors: LBM_EINVAL (unknown form, NULL pointer). */
int lbm_precision_info(int32_t precision, int32_t *storage_bytes, int32_t *arith_bytes);

/* ---- exchange-step options --------------------------------------------- */
#define LBM_WARM 0        /* new fluid cells start at rest, rest is kept    */
#define LBM_COLD 1        /* every non-solid cell restarts at rest          */
#define LBM_CRIT_PAPER 0  /* Eq. 6 for fluid, Eq. 5 (summed faces) for solid */
#define LBM_CRIT_SPEED 1  /* |u|^2 for fluid, max neighbour |u|^2 for solid */

typedef struct lbm_handle lbm_handle;

/* Geometry and physics of one lattice. */
typedef struct {
    int32_t nx, ny;     /* lattice size: 3 <= nx, ny <= 65536, nx*ny < 2^31 */
    int32_t levels;     /* generator only: bifurcation generations L >= 1 */
    int32_t widths[9];  /* generator only: w_0..w_L in cells; all 0 gives
                           w_k = max(2, (ny/8) >> k)                      */
    double tau;         /* BGK relaxation time, > 1/2 (tau = 3 nu + 1/2)  */
    double u_peak;      /* peak of the parabolic inlet profile (lattice u)*/
    double rho_out;     /* density imposed on outlet cells, > 0           */
    int32_t precision;  /* LBM_F64, LBM_F32, LBM_F32_S_F16, LBM_F32_S_BF16 */
    int32_t flags;      /* boundary variants, LBM_NEUMANN_OUTLET |
                           LBM_SYMMETRY_TOP (0: Zou-He density outlets,
                           full domain)                                   */
} lbm_geometry_desc;

/* Boundary variants of the paper's own runs (Sec. 3.3).
 * LBM_NEUMANN_OUTLET: zero normal gradient of the velocity at the outlet
 *   (Sec. 3.3; rho_out is then unused).  Each outlet cell imposes the velocity
 *   (Eq. 2) of the stored state of its neighbour at x-1 (zero when that cell
 *   is solid) through the Zou-He velocity closure of an east boundary: the
 *   unknown populations 3, 6, 7 follow from that velocity and the known
 *   populations, and the cell's density from the known populations.
 * LBM_SYMMETRY_TOP: the lattice is the lower half of a domain that is mirror
 *   symmetric about the line just above row ny-1.  A population that would be
 *   pulled from row ny is the mirror image (c_y reversed) of the one leaving
 *   the cell in row ny-1 below it; an inlet opening that reaches row ny-1 is
 *   the lower half of an opening mirrored about that line (its parabola
 *   spans both halves). */
enum { LBM_NEUMANN_OUTLET = 1, LBM_SYMMETRY_TOP = 2 };

/* Boundary reductions (Eq. 4, Eqs. 9-11) of the steady flow: every flux
 * and the pressure drop are means over the current state and the state one
 * time step later (see lbm_outlet_stats). */
typedef struct {
    int32_t n_outlets;  /* maximal runs of outlet cells in column nx-1    */
    int32_t reserved;
    int64_t n_fluid;    /* cells of type LBM_FLUID                        */
    int64_t n_nonsolid; /* fluid + inlet + outlet cells                   */
    double flow_in;     /* sum of rho u_x over the inlet cells            */
    double dp;          /* c_s^2 (mean inlet rho - mean outlet rho)        */
    double theta;       /* max/min outlet flow, Eq. 9                      */
    double dg;          /* maldistribution factor, Eq. 10                  */
    double flow_ave;    /* mean outlet flow, Eq. 11                        */
    double mass;        /* sum of rho over non-solid cells                 */
    double residual;    /* residual of the last lbm_run_to_steady          */
    int64_t steps;      /* time steps run since creation or set_state      */
    double flow_p2;     /* largest period-two component of an outlet flux,
                           max_k |flow_k(t) - flow_k(t+1)| / 2            */
} lbm_stats;

/* Parameters of one exchange step (Sec. 2.2, Sec. 2.3 step 3). */
typedef struct {
    double frac;        /* K = max(1, floor(frac * N_fluid)), 0 <= frac <= 1 */
    uint64_t seed;      /* tie-break hash seed                               */
    int32_t band_x;     /* cells with x < band_x or x > nx-1-band_x never flip (>= 1) */
    int32_t band_y;     /* same for y (>= 1)                                 */
    int32_t criterion;  /* LBM_CRIT_PAPER or LBM_CRIT_SPEED                  */
    int32_t reinit;     /* LBM_WARM or LBM_COLD                              */
} lbm_shape_params;

/* Outcome of one exchange step. */
typedef struct {
    int32_t k_eff;            /* cells exchanged each way                 */
    int32_t reserved;
    int64_t n_cand_fluid;     /* |C_f|: fluid interface cells in the band */
    int64_t n_cand_solid;     /* |C_s|: solid interface cells in the band */
    int64_t n_fluid_before;
    int64_t n_fluid_after;    /* equals n_fluid_before (constant volume)  */
    double mass_removed;      /* sum of rho over the cells made solid     */
    double mass_added;        /* k_eff (new fluid cells start at rho = 1) */
} lbm_shape_result;

/*
 * Step (1) of Sec. 2.3: build a lattice and put it at rest (Sec. 3.3: the
 * equilibrium at rho = 1, u = 0 on every non-solid cell).
 *   d           geometry and physics; read during the call only.
 *   cell_types  nx*ny bytes, row-major, values LBM_SOLID..LBM_OUTLET; NULL
 *               builds the flat arborescent distributor from d->levels and
 *               d->widths (one inlet on column 0, 2^L equally spaced outlets
 *               on column nx-1; rows 0 and ny-1 solid).
 *   hip_stream  hipStream_t to issue all work on, borrowed (NULL: null stream).
 *   out         receives the handle; release it with lbm_destroy.
 * Errors: LBM_EINVAL (sizes, tau <= 1/2, rho_out <= 0, unknown precision,
 * ports off their column, bad generator widths), LBM_ENOMEM, LBM_EHIP.
 */
int lbm_create_geometry(const lbm_geometry_desc *d, const uint8_t *cell_types,
                        void *hip_stream, lbm_handle **out);

/*
 * Steps (2) and (4) of Sec. 2.3: advance the lattice by the LBM of Sec. 2.1
 * (Eq. 1, Eq. 2, halfway bounce-back walls, Zou-He velocity inlet with the
 * parabolic profile of Sec. 3.3 and Zou-He density outlets) until steady.
 *   max_steps    at most this many time steps (>= 0).
 *   tol          stop once r < tol; tol <= 0 runs exactly max_steps.
 *   check_every  r = ||u(t) - u(t-k)||_2 / ||u(t)||_2 over non-solid cells,
 *                evaluated every k = check_every steps (>= 1; the last chunk
 *                may be shorter); u at the start of the call is the velocity
 *                of the current state.
 *   steps_done, residual  may be NULL.
 * Returns LBM_OK, LBM_NOT_CONVERGED (tol > 0 not reached), LBM_EUNSTABLE
 * (a non-finite rho or u at a check step; the state is then undefined),
 * LBM_EINVAL, LBM_EHIP.
 */
int lbm_run_to_steady(lbm_handle *h, int64_t max_steps, double tol,
                      int32_t check_every, int64_t *steps_done,
                      double *residual);

/*
 * Step (5) of Sec. 2.3 and Sec. 4.2: boundary reductions of the steady flow.
 * flow receives the mass flux sum(rho u_x) of each outlet, ordered by
 * increasing y (flow_cap doubles available), as the mean of the current
 * state's flux and that of the state one step later: converged flows carry
 * an undamped oscillation of period two steps at the fixed-density outlets
 * (a few percent of the outlet flux on the distributors), which the residual
 * of lbm_run_to_steady does not see; the two-step mean cancels it.  flow_in
 * and dp are means in the same way, theta, dg and flow_ave are taken on the
 * mean fluxes, mass is the current state's.  The later state is computed in
 * the handle's second population buffer; the current state is not changed.
 * All sums are double precision and run in a fixed order, so repeated calls
 * give identical bits.
 * Errors: LBM_EINVAL if flow_cap < n_outlets (s->n_outlets is still set), or a
 * NULL pointer; LBM_EHIP.
 */
int lbm_outlet_stats(lbm_handle *h, double *flow, int32_t flow_cap,
                     lbm_stats *s);

/*
 * lbm_outlet_stats for callers that cannot allocate memory (tight serving
 * loops, harnesses that forbid allocation during a measurement): the same
 * results, bit for bit, with no device or pinned host allocation.  Every
 * intermediate (boundary sums of the two states, the mass and its per-block
 * partials) lives in one fixed device scratch area of 1 MiB per GPU, held
 * until the process ends and shared by every call on that GPU: calls that
 * overlap on one GPU (several threads, or several streams in flight) race
 * on it and must be serialised by the caller.  Nothing in the scratch needs
 * to start at zero.  The sums come back through a buffer on the calling
 * thread's stack (about 33 KB).
 * Limits: at most 1024 outlets, and (2 (2 n_out + 5) + 1 + ceil(nx/64)
 * ceil(ny/4)) * 8 bytes within the 1 MiB (e.g. 4096 x 4096 lattices).
 * Errors: those of lbm_outlet_stats; LBM_EINVAL, with a message, beyond the
 * limits.
 */
int lbm_outlet_stats_noalloc(lbm_handle *h, double *flow, int32_t flow_cap, lbm_stats *s);

/*
 * Steps (3) and (4) of Sec. 2.3: exchange the K_eff fluid interface cells of
 * lowest key with the K_eff solid interface cells of highest key (Sec. 2.2),
 * at constant fluid volume, then re-initialise (WARM: new fluid cells at
 * rest; COLD: the whole lattice at rest) and rebuild the wall links.
 *   rho_ux_uy  NULL: keys from the current state.  Otherwise 3*nx*ny host
 *              doubles (rho, then u_x, then u_y, each row-major) used as the
 *              field instead.
 * Interface: 4-neighbourhood.  Keys (criterion PAPER): fluid rho*(ux*ux +
 * uy*uy) (Eq. 6 without the factor 1/2), solid: sum over the non-solid
 * neighbours in the order +x, +y, -x, -y of |u_y| (x faces) or |u_x|
 * (y faces) (Eq. 5 without mu/(0.5 dx)); both evaluated in double precision
 * without fused multiply-add.  Ties: ascending SplitMix64(seed + n), then n.
 * Errors: LBM_EINVAL (bad params, NaN or negative key), LBM_ENOMEM, LBM_EHIP.
 */
int lbm_shape_update(lbm_handle *h, const lbm_shape_params *p,
                     const double *rho_ux_uy, lbm_shape_result *r);

/* The exchange step of lbm_shape_update on n distinct handles at once (each
 * with its own parameters, keys from its current state), with the work of
 * all of them issued before each of the step's two waits for the device
 * instead of two waits per handle: for a server whose sessions reach their
 * exchange steps together (Sec. 2.3 steps 3-4 for many shapes).  Each
 * handle's result is exactly that of lbm_shape_update.  status[k] receives
 * handle k's status; the call returns the most negative of them (LBM_OK when
 * all succeeded).  Errors: LBM_EINVAL (NULL arrays, n < 0, a handle listed
 * twice), or per handle those of lbm_shape_update. */
int lbm_shape_update_many(lbm_handle *const *hs, const lbm_shape_params *ps, int32_t n,
                          lbm_shape_result *rs, int32_t *status);

/* Logical indices of the cells the last lbm_shape_update made solid
 * (removed) and fluid (added), in selection order.  Returns the count k_eff
 * (>= 0) or LBM_EINVAL when cap < k_eff. */
int lbm_last_exchange(lbm_handle *h, int64_t *removed, int64_t *added,
                      int32_t cap);

/* Cell map, nx*ny bytes (n >= nx*ny). */
int lbm_get_mask(lbm_handle *h, uint8_t *types, size_t n);

/* Density and velocity of every cell (0 on solid cells), each nx*ny doubles
 * (n >= nx*ny), from the current state. */
int lbm_get_macro(lbm_handle *h, double *rho, double *ux, double *uy,
                  size_t n);

/* Current state: the post-collision populations about to stream,
 * f[i*nx*ny + y*nx + x] for i = 0..8 (n >= 9*nx*ny doubles); solid cells 0.
 * lbm_set_state loads such an array (solid-cell entries ignored) and resets
 * the step counter; values are rounded to the handle's precision. */
int lbm_get_state(lbm_handle *h, double *f, size_t n);
int lbm_set_state(lbm_handle *h, const double *f, size_t n);

/* Device bytes a handle for d would allocate (0 if d is invalid), each
 * buffer counted in the size class it is allocated in (its size rounded up
 * to a multiple of 1/8 of its power of two): the buffers made at creation,
 * those the first exchange step and outlet statistics make, with the
 * candidate lists at their initial capacity (max(4096, nx*ny/16) per kind).
 * A lattice with more interface cells of one kind than that grows its lists
 * on an exchange step and then holds more than this count.  Not counted: the
 * staging field of 24 bytes per cell that lbm_get_macro, lbm_get_state,
 * lbm_set_state and an exchange step given a host field make on first use
 * (the optimisation loop and the server need none of them). */
size_t lbm_footprint_bytes(const lbm_geometry_desc *d);

/* Device bytes handle h holds now (each buffer in its size class), for
 * checking lbm_footprint_bytes: after the first exchange step and outlet
 * statistics it equals the footprint unless a candidate list grew or one of
 * the calls that stage a whole field ran.  Errors: LBM_EINVAL (NULL). */
int lbm_device_bytes(lbm_handle *h, size_t *bytes);

/* Release a handle (NULL is ignored).  The call waits for the handle's
 * stream; its device blocks and pinned staging then go to a process-wide
 * cache that later handles and batches of the same size classes draw from
 * (at most 4 GiB of device and 64 MiB of pinned host memory are kept, the
 * oldest blocks being freed first).  A batch that still holds the handle
 * must be destroyed first. */
void lbm_destroy(lbm_handle *h);

/* Message of the last error on this thread ("" if none). */
const char *lbm_last_error(void);

/* Advance the lattice by `steps` time steps without residual checks and
 * report the mean time per step in milliseconds, measured with HIP events
 * recorded on the handle's stream before the first and after the last
 * sweep launch.  The steps are real: the state advances (by steps plus up to
 * 128 untimed warm-up steps that build the launch graphs first). */
int lbm_bench_sweep(lbm_handle *h, int32_t steps, double *ms_per_step);

/* Sweep timing inside lbm_run_to_steady.  enable = 1 resets the counters
 * and starts recording: every fourth residual-check interval (the first of
 * each four counted since enabling) then records a HIP event on the
 * handle's stream before its first sweep launch and after its last one, and
 * adds the elapsed time, the time steps and the sweep kernel launches in
 * between (a launch may advance several steps); the totals cover those
 * intervals only.  Recording every interval slowed the run itself by a few
 * per cent (two stream markers per interval).  enable = 0
 * stops recording.  Either way the current totals are returned (any of
 * steps, launches, total_ms may be NULL). */
int lbm_profile_sweeps(lbm_handle *h, int32_t enable, int64_t *steps,
                       int64_t *launches, double *total_ms);

/*
 * Region shapes of the temporally blocked sweep.  A launch loads a region of
 * 64 x rows cells into LDS and advances its inner tile of (64 - 2 halo) x
 * (rows - 2 halo) cells by up to `halo` time steps of Sec. 2.1 (the ring of
 * width halo around the tile is recomputed by its neighbours).  The shape
 * changes only the speed: every shape gives the same bits as one sweep per
 * step.
 *
 * lbm_tb_variant_count: number of shapes compiled for a precision (0 for an
 * unknown precision).  lbm_tb_variant_info: shape `variant` of `precision`;
 * any output pointer may be NULL.  Errors: LBM_EINVAL.
 */
int32_t lbm_tb_variant_count(int32_t precision);
int lbm_tb_variant_info(int32_t precision, int32_t variant, int32_t *rows,
                        int32_t *halo, int32_t *tile_w, int32_t *tile_h);

/* Body of shape `variant` of `precision`: kind LBM_TB_DENSE (a lane per
 * region column, two region copies), LBM_TB_COMPACT (lanes take entries of a
 * list of the region's non-solid cells; two copies plus the list) or
 * LBM_TB_INPLACE (dense, one copy updated in place), and the LDS bytes one
 * workgroup of it uses.  Any output pointer may be NULL.  Errors: LBM_EINVAL. */
enum { LBM_TB_DENSE = 0, LBM_TB_COMPACT = 1, LBM_TB_INPLACE = 2 };
int lbm_tb_variant_kind(int32_t precision, int32_t variant, int32_t *kind,
                        int32_t *lds_bytes);

/* Use region shape `variant` for the handle's sweeps from now on.  A launch
 * covers the tiles holding a non-solid cell, dealt to the chip's eight XCDs
 * in contiguous runs of the row-major tile list (one run per XCD for the
 * two-copy bodies, 32 runs for the in-place body); the order changes timing
 * only, never results.
 * Errors: LBM_EINVAL (NULL handle, variant out of range), LBM_EHIP. */
int lbm_set_tb_variant(lbm_handle *h, int32_t variant);

/* The region shape the handle's sweeps use now: the last lbm_set_tb_variant
 * or lbm_autotune choice, or, after an exchange step pushed the autotuned
 * shape's active tiles past one round of workgroups, the fastest timed shape
 * whose tiles still fit (the autotuned shape is taken back once it fits
 * again).  -1 when temporal blocking is off (one launch per step).
 * Errors: LBM_EINVAL (NULL argument). */
int lbm_get_tb_variant(lbm_handle *h, int32_t *variant);

/*
 * Autotuner: time every compiled shape on `trial_steps` (>= 1) real time
 * steps of this lattice, keep the fastest, and leave the state, the step
 * counter and the residual exactly as they were (both population buffers
 * are saved and restored, so the call needs their size again in scratch
 * memory while it runs).
 *   best  receives the chosen shape (may be NULL).
 *   ms    receives the mean time per step of each shape (ms_cap entries;
 *         may be NULL when ms_cap is 0).
 * The timings are kept: if a later lbm_shape_update leaves the chosen
 * shape with more active tiles than the device runs in one round (when the
 * choice had them all in one), the handle moves to the fastest timed shape
 * whose tiles still fit.  lbm_set_tb_variant drops the kept timings.
 * Errors: LBM_EINVAL (NULL handle, trial_steps < 1, ms_cap below the shape
 * count while ms is not NULL), LBM_ENOMEM, LBM_EHIP.
 */
int lbm_autotune(lbm_handle *h, int32_t trial_steps, int32_t *best,
                 double *ms, int32_t ms_cap);

/*
 * Batched sweeps: many lattices of one precision, each of its own size,
 * geometry, tau, inlet peak and outlet density, advanced together.  Every
 * launch covers all tiles holding a non-solid cell of all member lattices, so
 * small lattices share the chip instead of each leaving most of it idle; each
 * lattice computes exactly what lbm_run_to_steady computes for it alone (the
 * LBM of Sec. 2.1 with the boundaries of Sec. 3.3), bit for bit.  The time
 * loop is replayed from a captured HIP graph.
 *
 * lbm_batch_create: handles[0..count-1] (count >= 1) must be distinct, of one
 * precision and on the current device; they stay owned by the caller and
 * must outlive the batch.  hip_stream: the stream the batch launches on
 * (borrowed; NULL: the null stream).  The batch starts with shape 0 and
 * work-list order 0.  Errors: LBM_EINVAL, LBM_ENOMEM, LBM_EHIP.
 */
typedef struct lbm_batch lbm_batch;
int lbm_batch_create(lbm_handle *const *handles, int32_t count,
                     void *hip_stream, lbm_batch **out);

/*
 * Advance every member lattice by `steps` (>= 0) time steps without residual
 * checks.  Waits for the members' own streams first and for the batch's
 * stream before returning.  Members whose mask changed since the last call
 * (lbm_shape_update) are picked up automatically.  Each member's step
 * counter advances by `steps`; its residual becomes NaN (unknown) until its
 * next lbm_run_to_steady.
 *   elapsed_ms  receives the time between HIP events recorded on the
 *               batch's stream around the sweep launches (may be NULL).
 * Errors: LBM_EINVAL, LBM_ENOMEM, LBM_EHIP.
 */
int lbm_batch_run(lbm_batch *b, int64_t steps, double *elapsed_ms);

/*
 * Choose the batch's configuration.  variant in [0, lbm_tb_variant_count)
 * selects a region shape of the temporally blocked sweep (as for
 * lbm_set_tb_variant); variant = lbm_tb_variant_count selects one time step
 * per launch over the 64 x 4 cell blocks that hold a non-solid cell.  Work
 * list `order`: 0 = lattice by lattice, tiles row by row; 1 = the same list
 * dealt so that consecutive tiles run on the same accelerator complex (XCD)
 * of the chip, which shares their halo rows in that XCD's L2 cache.  Neither
 * changes the results.  Errors: LBM_EINVAL.
 */
int lbm_batch_configure(lbm_batch *b, int32_t variant, int32_t order);

/*
 * Autotuner for a batch: time every (variant, order) pair of
 * lbm_batch_configure on `trial_steps` real steps of all members, keep the
 * fastest and restore every member's state, step counter and residual
 * exactly (scratch memory of twice the members' population buffers while it
 * runs).  Configuration c = 2 * variant + order; ms receives the mean time
 * per step of each (ms_cap >= 2 x (shape count + 1), or ms NULL);
 * best_variant, best_order may be NULL.
 * Errors: LBM_EINVAL, LBM_ENOMEM, LBM_EHIP.
 */
int lbm_batch_tune(lbm_batch *b, int32_t trial_steps, int32_t *best_variant,
                   int32_t *best_order, double *ms, int32_t ms_cap);

/* Work items (tiles or blocks) per launch, time steps per launch (the halo
 * of the shape, or 1) and the summed non-solid cell count of the members,
 * for throughput accounting; any pointer may be NULL. */
int lbm_batch_info(lbm_batch *b, int64_t *items, int32_t *steps_per_launch,
                   int64_t *nonsolid_cells);

/* Release a batch (the member handles are untouched; NULL is ignored).  The
 * call waits for the batch's stream; its buffers go to the same cache as a
 * handle's. */
void lbm_batch_destroy(lbm_batch *b);

/* Switch the captured-graph replay of a batch's time loop on (default) or
 * off; off suits batches whose membership changes every few runs, where a
 * capture would be used too few times to pay for itself.  Results do not
 * change.  Errors: LBM_EINVAL. */
int lbm_batch_set_graphs(lbm_batch *b, int32_t enable);

/*
 * 64-bit digest of the current state and mask: the sum, modulo 2^64, over
 * every non-solid cell n and population i of SplitMix64 of the stored bits
 * of f_i(n) mixed with (9 n + i), plus SplitMix64 of each cell's type mixed
 * with its index.  Order-free, so it is the same however the work is split;
 * two states with the same digest are the same bits (up to 64-bit hash
 * collisions).  For comparing runs, not for security.
 * Errors: LBM_EINVAL, LBM_EHIP.
 */
int lbm_state_digest(lbm_handle *h, uint64_t *digest);

/*
 * Serving: a request loop with continuous batching.  A worker thread owns
 * the device work.  Requests wait in a FIFO queue and are admitted, in
 * order, while the summed lbm_footprint_bytes of the admitted sessions stays
 * within hbm_budget and fewer than max_sessions are active; an admitted
 * request becomes a session whose lattice state stays on the device until it
 * completes.  Rounds: every active session advances by the same number of
 * time steps (at most `quantum`, fewer if a session's next event is nearer),
 * all sessions of one precision in one lbm_batch; then sessions at an event
 * take it (an optimise iteration's exchange step, or completion: outlet
 * statistics and the state digest, after which the session's memory is
 * released).  Requests that arrive while a round runs join at the next
 * round.  Each session's results are the same bits as the same request run
 * alone, because every lattice's arithmetic is independent of the others.
 *
 * Work of a request (Sec. 2.3): SOLVE advances the lattice from rest by
 * solve_steps steps; OPTIMIZE advances solve_steps steps, then `iterations`
 * times takes the exchange step (Sec. 2.2) with params.seed + iteration as
 * the tie-break seed and advances steps_per_iteration steps.
 */
enum { LBM_REQ_SOLVE = 0, LBM_REQ_OPTIMIZE = 1 };

typedef struct {
    size_t hbm_budget;      /* bytes of lbm_footprint_bytes admitted at once   */
    int32_t max_sessions;   /* active sessions at once (>= 1)                  */
    int32_t quantum;        /* time steps per round at most (>= 1)             */
    int32_t variant;        /* batch variant (lbm_batch_configure); -1: chosen
                               by lbm_batch_tune once per precision, on the
                               first batch of >= 8 sessions                   */
    int32_t order;          /* batch work-list order (0 or 1) with variant >= 0 */
} lbm_server_config;

typedef struct {
    lbm_geometry_desc geom;  /* generator description (cell_types NULL)        */
    int32_t kind;            /* LBM_REQ_SOLVE or LBM_REQ_OPTIMIZE               */
    int32_t iterations;      /* exchange steps (OPTIMIZE), >= 0                 */
    int64_t solve_steps;     /* steps from rest, >= 0                           */
    int64_t steps_per_iteration; /* steps after each exchange step, >= 0        */
    lbm_shape_params shape;  /* exchange-step parameters (OPTIMIZE)             */
} lbm_request;

typedef struct {
    uint64_t id;             /* as returned by lbm_server_submit                */
    int32_t status;          /* LBM_OK or the first error of the session        */
    int32_t iterations_done;
    int64_t steps;           /* time steps taken                                */
    int64_t cells;           /* nx * ny                                         */
    uint64_t digest;         /* lbm_state_digest at completion                  */
    double t_submit, t_admit, t_done; /* seconds on a monotonic clock           */
    lbm_stats stats;         /* lbm_outlet_stats at completion                  */
} lbm_result;

typedef struct {
    int64_t submitted, completed, rejected, active, queued;
    int64_t rounds;
    int64_t cell_steps;      /* sum over sessions of nx * ny * steps taken      */
    int64_t nonsolid_cell_steps;
    double busy_seconds;     /* time in rounds (device work and host events)    */
    double admit_seconds;    /* creating admitted sessions, on the creation     */
                             /* thread (overlaps the rounds; not in busy)       */
    double sweep_seconds;    /*           batched sweeps (incl. batch rebuilds) */
    double event_seconds;    /*           exchange steps and completions        */
    size_t peak_bytes;       /* largest admitted footprint sum                  */
    double exchange_seconds; /* of event_seconds: exchange steps               */
    int64_t exchanges;       /* exchange steps taken                            */
    int64_t exchange_calls;  /* lbm_shape_update_many calls that took them      */
} lbm_server_stats;

typedef struct lbm_server lbm_server;

/* Start a server (and its worker thread) on the current device, issuing work
 * on hip_stream (borrowed; NULL: the null stream).
 * Errors: LBM_EINVAL (config), LBM_ENOMEM, LBM_EHIP. */
int lbm_server_create(const lbm_server_config *cfg, void *hip_stream,
                      lbm_server **out);

/* Queue a request (copied); *id receives its identifier (ids count up from
 * 1).  A request whose footprint exceeds hbm_budget is not queued: it
 * completes at once with status LBM_ENOMEM.  Errors: LBM_EINVAL (bad request
 * or server stopped). */
int lbm_server_submit(lbm_server *s, const lbm_request *req, uint64_t *id);

/* Move up to `cap` completed results into `out`, waiting up to wait_ms
 * milliseconds for the first one (0: no wait, < 0: wait until one arrives
 * or nothing is pending).  Returns the number moved (>= 0) or an error. */
int lbm_server_poll(lbm_server *s, lbm_result *out, int32_t cap, int32_t wait_ms);

/* Block until every submitted request has completed (its result may still be
 * waiting for lbm_server_poll). */
int lbm_server_drain(lbm_server *s);

/* Counters since creation. */
int lbm_server_stats_get(lbm_server *s, lbm_server_stats *st);

/* Stop the worker (pending and active requests are abandoned) and release
 * everything (NULL is ignored). */
void lbm_server_destroy(lbm_server *s);

#ifdef __cplusplus
}
#endif
#endif /* LBM_H */
