/*
 * FP64 CPU oracle for the lattice-Boltzmann shape-optimisation method of
 * Wang, Fan & Luo, "Lattice Boltzmann method for shape optimization of fluid
 * distributor" (Computers & Fluids).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously correct
 * statement of what the GPU path computes.  Only the test-suite, the smoke
 * check and the CPU-baseline leg of the benchmark may load it.  It shares no
 * code, header, table or constant with the HIP library and includes nothing
 * from it.
 *
 * Build: gcc -O2 -ffp-contract=off -fopenmp -shared -fPIC (no FMA contraction,
 * so every expression is evaluated exactly in the order written).  OpenMP only
 * splits independent per-cell loops over rows; every reduction is a single
 * sequential loop in row-major order, so the result does not depend on the
 * thread count.
 *
 * Conventions
 *   - Lattice nx x ny, cell (x, y) at index n = y*nx + x (row-major, y outer).
 *   - Cell types: 0 solid, 1 fluid, 2 inlet, 3 outlet (Sec. 3.3, Fig. 5).
 *   - Populations are stored plane-major: f[i*N + n], N = nx*ny.
 *   - The state handed in and out (`fs`) is the post-collision population set,
 *     i.e. the values that are about to stream.  BGK collision conserves mass
 *     and momentum, so the density and velocity of this state are those of the
 *     pre-collision state it was relaxed from.
 *   - Solid cells carry zero populations.
 *
 * One time step (Sec. 2.1, Eq. 1):
 *   1. stream (pull) with halfway bounce-back at solid / out-of-domain sources;
 *   2. boundary conditions on inlet and outlet cells (Sec. 3.3: parabolic
 *      velocity inlet; outlets at fixed density), imposed with the Zou-He
 *      non-equilibrium bounce-back construction;
 *      or, as the paper's own runs (Sec. 3.3), a zero-gradient (Neumann)
 *      outlet and a symmetry plane that halves the domain (flags below);
 *   3. moments rho, u (Eq. 2);
 *   4. BGK relaxation towards the second-order equilibrium (Eq. 1 and the
 *      equilibrium of Sec. 2.1).
 */
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define Q 9

enum { T_SOLID = 0, T_FLUID = 1, T_INLET = 2, T_OUTLET = 3 };
/* Boundary variants of Sec. 3.3 (bit flags):
 *   ORC_NEUMANN_OUTLET  zero normal gradient of the velocity at the outlet:
 *                       each outlet cell imposes the velocity (Eq. 2) of the
 *                       stored state of its neighbour at x-1 (zero if that
 *                       cell is solid) with the Zou-He velocity closure of an
 *                       east boundary, instead of a fixed density;
 *   ORC_SYMMETRY_TOP    the lattice is the lower half of a domain symmetric
 *                       about the line just above row ny-1: a population
 *                       pulled from row ny is the mirror image (c_y reversed)
 *                       of the one leaving the cell below it in row ny-1. */
enum { ORC_NEUMANN_OUTLET = 1, ORC_SYMMETRY_TOP = 2 };
enum {
    ORC_OK = 0,
    ORC_NOT_CONVERGED = 1,
    ORC_EINVAL = -1,
    ORC_ENOMEM = -2,
    ORC_EUNSTABLE = -4
};

/* D2Q9 velocity set, Sec. 2.1: c0 = 0; c1..c4 = (cos, sin) of (i-1)*pi/2;
 * c5..c8 are the diagonals at 45 + (i-5)*90 degrees with length sqrt(2)
 * (the printed angle formula for i = 5..8 drops the 45-degree offset). */
static const int CX[Q] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int CY[Q] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
/* index of -c_i */
static const int OPP[Q] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
/* index of the mirror image of c_i under y -> -y */
static const int MIRY[Q] = {0, 1, 4, 3, 2, 8, 7, 6, 5};
/* weights 4/9, 1/9 (i = 1..4), 1/36 (i = 5..8), Sec. 2.1 */
static const double WT[Q] = {4.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0,
                             1.0 / 9.0,  1.0 / 9.0,  1.0 / 36.0,
                             1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
/* 1/c_s^2 with c_s = sqrt(3)/3 in lattice units (Sec. 2.1) */
static const double INV_CS2 = 3.0;

void orc_velocity_set(int *cx, int *cy, int *opp, double *w) {
    for (int i = 0; i < Q; ++i) {
        cx[i] = CX[i];
        cy[i] = CY[i];
        opp[i] = OPP[i];
        w[i] = WT[i];
    }
}

/* Equilibrium of Sec. 2.1:
 * feq_i = w_i rho (1 + c.u/cs^2 + (c.u)^2/(2 cs^4) - u.u/(2 cs^2)). */
void orc_equilibrium(double rho, double ux, double uy, double *feq) {
    double uu = ux * ux + uy * uy;
    for (int i = 0; i < Q; ++i) {
        double cu = CX[i] * ux + CY[i] * uy;
        feq[i] = WT[i] * rho *
                 (1.0 + cu * INV_CS2 + 0.5 * (cu * cu) * (INV_CS2 * INV_CS2) -
                  0.5 * uu * INV_CS2);
    }
}

/* Moments of Eq. 2, summed in index order. */
static void moments9(const double *f, double *rho, double *jx, double *jy) {
    double r = 0.0, mx = 0.0, my = 0.0;
    for (int i = 0; i < Q; ++i) {
        r += f[i];
        mx += CX[i] * f[i];
        my += CY[i] * f[i];
    }
    *rho = r;
    *jx = mx;
    *jy = my;
}

/* BGK relaxation of Eq. 1 for one cell: f* = f - (1/tau)(f - feq). */
void orc_collide_cell(const double *f, double tau, double *fout) {
    double rho, jx, jy, feq[Q];
    const double omega = 1.0 / tau;
    moments9(f, &rho, &jx, &jy);
    orc_equilibrium(rho, jx / rho, jy / rho, feq);
    for (int i = 0; i < Q; ++i) fout[i] = f[i] - omega * (f[i] - feq[i]);
}

/* tau = 3 nu + dt/2 with dt = 1 (Sec. 2.1). */
double orc_tau_from_nu(double nu) { return 3.0 * nu + 0.5; }

/* Parabolic inlet profile (Sec. 3.3) on every maximal run of inlet cells in
 * column 0: rows y0..y1, walls half a cell outside the run,
 * u(y) = 4 u_peak [(y - y0 + 1/2)(y1 + 1/2 - y)] / W^2, W = y1 - y0 + 1.
 * With ORC_SYMMETRY_TOP a run that reaches row ny-1 is the lower half of an
 * opening mirrored about the symmetry line: y1 = 2 ny - 1 - y0.
 * The product of the two wall distances is formed first, so rows mirrored
 * about the centre of the opening get bitwise equal values.
 * Rows that are not inlet cells get 0. */
void orc_inlet_profile_ex(int nx, int ny, const uint8_t *type, double u_peak,
                          int32_t flags, double *uin) {
    for (int y = 0; y < ny; ++y) uin[y] = 0.0;
    int y = 0;
    while (y < ny) {
        if (type[(size_t)y * nx] != T_INLET) {
            ++y;
            continue;
        }
        int y0 = y;
        while (y < ny && type[(size_t)y * nx] == T_INLET) ++y;
        int last = y - 1;
        int y1 = last;
        if ((flags & ORC_SYMMETRY_TOP) && last == ny - 1) y1 = 2 * ny - 1 - y0;
        double W = (double)(y1 - y0 + 1);
        for (int r = y0; r <= last; ++r) {
            double a = (double)(r - y0) + 0.5;
            double b = (double)(y1 - r) + 0.5;
            uin[r] = 4.0 * u_peak * (a * b) / (W * W);
        }
    }
}

void orc_inlet_profile(int nx, int ny, const uint8_t *type, double u_peak,
                       double *uin) {
    orc_inlet_profile_ex(nx, ny, type, u_peak, 0, uin);
}

/* Input checks shared by every entry point of this file. */
static int check_types(int nx, int ny, const uint8_t *type) {
    if (nx < 2 || ny < 1) return ORC_EINVAL;
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            uint8_t t = type[(size_t)y * nx + x];
            if (t > T_OUTLET) return ORC_EINVAL;
            if (t == T_INLET && x != 0) return ORC_EINVAL;
            if (t == T_OUTLET && x != nx - 1) return ORC_EINVAL;
        }
    return ORC_OK;
}

/* Pass 1: pull streaming, Eq. 1: f_i(x) <- fs_i(x - c_i).  If x - c_i is
 * solid or outside the lattice, the link is cut by a wall halfway between the
 * two nodes, and the population that left x towards that wall, fs_opp(i)(x),
 * returns reversed (no-slip, Sec. 3.3).  With ORC_SYMMETRY_TOP a source in
 * row ny (just beyond the symmetry line) stands for the mirror image of row
 * ny-1: fs_mirror(i) at (x - cx_i, ny-1) (a wall if that cell is solid or off
 * the lattice). */
static double pull(int nx, int ny, const uint8_t *type, const double *fs,
                   int32_t flags, int x, int y, int i) {
    const size_t N = (size_t)nx * ny;
    const size_t n = (size_t)y * nx + x;
    int sx = x - CX[i], sy = y - CY[i], pop = i;
    if ((flags & ORC_SYMMETRY_TOP) && sy == ny) {
        sy = ny - 1;
        pop = MIRY[i];
    }
    int wall = sx < 0 || sx >= nx || sy < 0 || sy >= ny ||
               type[(size_t)sy * nx + sx] == T_SOLID;
    if (wall) return fs[OPP[i] * N + n];
    return fs[pop * N + (size_t)sy * nx + sx];
}

static void stream_pass(int nx, int ny, const uint8_t *type, const double *fs,
                        int32_t flags, double *f) {
    const size_t N = (size_t)nx * ny;
#pragma omp parallel for schedule(static)
    for (int y = 0; y < ny; ++y) {
        for (int x = 0; x < nx; ++x) {
            size_t n = (size_t)y * nx + x;
            if (type[n] == T_SOLID) {
                for (int i = 0; i < Q; ++i) f[i * N + n] = 0.0;
                continue;
            }
            for (int i = 0; i < Q; ++i) f[i * N + n] = pull(nx, ny, type, fs, flags, x, y, i);
        }
    }
}

/* Pass 2: boundary cells.
 * Inlet (x = 0): velocity (uin(y), 0) imposed; unknowns f1, f5, f8.
 * Outlet (x = nx-1): density rho_out and zero transverse velocity imposed;
 * unknowns f3, f6, f7.  With ORC_NEUMANN_OUTLET the outlet imposes instead
 * the velocity (ux, uy) of the stored state fs at (nx-2, y), and its density
 * follows from the known populations.  The known populations (including any
 * that came from a bounce-back link at the end of an opening) are used as
 * they are. */
static void boundary_pass(int nx, int ny, const uint8_t *type, const double *fs,
                          const double *uin, double rho_out, int32_t flags, double *f) {
    const size_t N = (size_t)nx * ny;
    for (int y = 0; y < ny; ++y) {
        size_t n = (size_t)y * nx;
        if (type[n] == T_INLET) {
            double ux = uin[y];
            double f0 = f[0 * N + n], f2 = f[2 * N + n], f3 = f[3 * N + n];
            double f4 = f[4 * N + n], f6 = f[6 * N + n], f7 = f[7 * N + n];
            double rho = (f0 + f2 + f4 + 2.0 * (f3 + f6 + f7)) / (1.0 - ux);
            double ru = rho * ux;
            f[1 * N + n] = f3 + (2.0 / 3.0) * ru;
            f[5 * N + n] = f7 - 0.5 * (f2 - f4) + (1.0 / 6.0) * ru;
            f[8 * N + n] = f6 + 0.5 * (f2 - f4) + (1.0 / 6.0) * ru;
        }
        n = (size_t)y * nx + (nx - 1);
        if (type[n] != T_OUTLET) continue;
        double f0 = f[0 * N + n], f1 = f[1 * N + n], f2 = f[2 * N + n];
        double f4 = f[4 * N + n], f5 = f[5 * N + n], f8 = f[8 * N + n];
        if (flags & ORC_NEUMANN_OUTLET) {
            double ux = 0.0, uy = 0.0;
            if (nx >= 2 && type[n - 1] != T_SOLID) {
                double fc[Q], r, jx, jy;
                for (int i = 0; i < Q; ++i) fc[i] = fs[i * N + n - 1];
                moments9(fc, &r, &jx, &jy);
                ux = jx / r;
                uy = jy / r;
            }
            double rho = (f0 + f2 + f4 + 2.0 * (f1 + f5 + f8)) / (1.0 + ux);
            double ru = rho * ux, rv = rho * uy;
            f[3 * N + n] = f1 - (2.0 / 3.0) * ru;
            f[7 * N + n] = f5 + 0.5 * (f2 - f4) - (1.0 / 6.0) * ru - 0.5 * rv;
            f[6 * N + n] = f8 - 0.5 * (f2 - f4) - (1.0 / 6.0) * ru + 0.5 * rv;
        } else {
            double ux = -1.0 + (f0 + f2 + f4 + 2.0 * (f1 + f5 + f8)) / rho_out;
            double ru = rho_out * ux;
            f[3 * N + n] = f1 - (2.0 / 3.0) * ru;
            f[7 * N + n] = f5 + 0.5 * (f2 - f4) - (1.0 / 6.0) * ru;
            f[6 * N + n] = f8 - 0.5 * (f2 - f4) - (1.0 / 6.0) * ru;
        }
    }
}

/* Pass 3: moments (Eq. 2) of every non-solid cell. */
static void moments_pass(int nx, int ny, const uint8_t *type, const double *f,
                         double *rho, double *ux, double *uy) {
    const size_t N = (size_t)nx * ny;
#pragma omp parallel for schedule(static)
    for (int y = 0; y < ny; ++y) {
        for (int x = 0; x < nx; ++x) {
            size_t n = (size_t)y * nx + x;
            if (type[n] == T_SOLID) {
                rho[n] = 0.0;
                ux[n] = 0.0;
                uy[n] = 0.0;
                continue;
            }
            double fc[Q], r, jx, jy;
            for (int i = 0; i < Q; ++i) fc[i] = f[i * N + n];
            moments9(fc, &r, &jx, &jy);
            rho[n] = r;
            ux[n] = jx / r;
            uy[n] = jy / r;
        }
    }
}

/* Pass 4: BGK relaxation (Eq. 1), f* = f - (1/tau)(f - feq), into fs. */
static void collide_pass(int nx, int ny, const uint8_t *type, const double *f,
                         const double *rho, const double *ux, const double *uy,
                         double tau, double *fs) {
    const size_t N = (size_t)nx * ny;
    const double omega = 1.0 / tau;
#pragma omp parallel for schedule(static)
    for (int y = 0; y < ny; ++y) {
        for (int x = 0; x < nx; ++x) {
            size_t n = (size_t)y * nx + x;
            if (type[n] == T_SOLID) {
                for (int i = 0; i < Q; ++i) fs[i * N + n] = 0.0;
                continue;
            }
            double feq[Q];
            orc_equilibrium(rho[n], ux[n], uy[n], feq);
            for (int i = 0; i < Q; ++i) {
                double fi = f[i * N + n];
                fs[i * N + n] = fi - omega * (fi - feq[i]);
            }
        }
    }
}

/* Residual r = ||u - u_prev||_2 / ||u||_2 over non-solid cells (the
 * steady-state test of Sec. 2.3 step (2): the flow field has stopped
 * changing), summed sequentially in row-major order.  A zero denominator
 * gives 0 when the numerator is zero too, +inf otherwise.  Exported so that
 * the tests can pin it on fields with a closed-form answer; orc_run_ex uses
 * this same function. */
double orc_residual(int nx, int ny, const uint8_t *type, const double *ux,
                    const double *uy, const double *pux, const double *puy) {
    const size_t N = (size_t)nx * ny;
    double num = 0.0, den = 0.0;
    for (size_t n = 0; n < N; ++n) {
        if (type[n] == T_SOLID) continue;
        double dx = ux[n] - pux[n], dy = uy[n] - puy[n];
        num += dx * dx + dy * dy;
        den += ux[n] * ux[n] + uy[n] * uy[n];
    }
    if (den == 0.0) return num == 0.0 ? 0.0 : INFINITY;
    return sqrt(num) / sqrt(den);
}

static int all_finite(int nx, int ny, const uint8_t *type, const double *rho,
                      const double *ux, const double *uy) {
    const size_t N = (size_t)nx * ny;
    for (size_t n = 0; n < N; ++n) {
        if (type[n] == T_SOLID) continue;
        if (!isfinite(rho[n]) || !isfinite(ux[n]) || !isfinite(uy[n]))
            return 0;
    }
    return 1;
}

/* Moments of the stored (post-collision) state. */
int orc_macro(int nx, int ny, const uint8_t *type, const double *fs,
              double *rho, double *ux, double *uy) {
    if (check_types(nx, ny, type) != ORC_OK) return ORC_EINVAL;
    moments_pass(nx, ny, type, fs, rho, ux, uy);
    return ORC_OK;
}

/* Initial condition of Sec. 3.3: equilibrium at rho0 = 1, u = 0, i.e.
 * f_i = w_i on every non-solid cell; solid cells hold zeros. */
int orc_init(int nx, int ny, const uint8_t *type, double *fs) {
    if (check_types(nx, ny, type) != ORC_OK) return ORC_EINVAL;
    const size_t N = (size_t)nx * ny;
    for (size_t n = 0; n < N; ++n)
        for (int i = 0; i < Q; ++i)
            fs[i * N + n] = type[n] == T_SOLID ? 0.0 : WT[i];
    return ORC_OK;
}

/*
 * Advance the state `fs` in place.
 *   max_steps   steps to run at most;
 *   tol         stop once the residual drops below tol (tol <= 0: run all);
 *   check_every the residual compares u with u from check_every steps
 *               earlier (the last chunk may be shorter); u at the start is the
 *               velocity of the state passed in;
 *   collide     0 skips relaxation (stream + boundary only) for tests.
 * Returns ORC_OK, ORC_NOT_CONVERGED (tol > 0 not reached) or ORC_EUNSTABLE
 * (a non-finite density or velocity at a check step).
 */
int orc_run_ex(int nx, int ny, const uint8_t *type, double tau, double u_peak,
               double rho_out, int32_t flags, double *fs, int64_t max_steps, double tol,
               int32_t check_every, int32_t collide, int64_t *steps_done,
               double *res_out) {
    if (check_types(nx, ny, type) != ORC_OK) return ORC_EINVAL;
    if (!(tau > 0.5) || check_every < 1 || max_steps < 0 || !(rho_out > 0.0))
        return ORC_EINVAL;
    if (flags & ~(ORC_NEUMANN_OUTLET | ORC_SYMMETRY_TOP)) return ORC_EINVAL;
    const size_t N = (size_t)nx * ny;
    double *f = malloc(sizeof(double) * Q * N);
    double *rho = malloc(sizeof(double) * N);
    double *ux = malloc(sizeof(double) * N);
    double *uy = malloc(sizeof(double) * N);
    double *pux = malloc(sizeof(double) * N);
    double *puy = malloc(sizeof(double) * N);
    double *uin = malloc(sizeof(double) * ny);
    int status = ORC_OK;
    if (!f || !rho || !ux || !uy || !pux || !puy || !uin) {
        status = ORC_ENOMEM;
        goto out;
    }
    orc_inlet_profile_ex(nx, ny, type, u_peak, flags, uin);
    moments_pass(nx, ny, type, fs, rho, pux, puy);
    int64_t done = 0;
    double res = 0.0;
    while (done < max_steps) {
        int64_t chunk = max_steps - done;
        if (chunk > check_every) chunk = check_every;
        for (int64_t s = 0; s < chunk; ++s) {
            stream_pass(nx, ny, type, fs, flags, f);
            boundary_pass(nx, ny, type, fs, uin, rho_out, flags, f);
            moments_pass(nx, ny, type, f, rho, ux, uy);
            if (collide)
                collide_pass(nx, ny, type, f, rho, ux, uy, tau, fs);
            else
                memcpy(fs, f, sizeof(double) * Q * N);
        }
        done += chunk;
        if (!all_finite(nx, ny, type, rho, ux, uy)) {
            status = ORC_EUNSTABLE;
            res = NAN;
            break;
        }
        res = orc_residual(nx, ny, type, ux, uy, pux, puy);
        memcpy(pux, ux, sizeof(double) * N);
        memcpy(puy, uy, sizeof(double) * N);
        if (tol > 0.0 && res < tol) break;
    }
    if (status == ORC_OK && tol > 0.0 && !(res < tol)) status = ORC_NOT_CONVERGED;
    if (steps_done) *steps_done = done;
    if (res_out) *res_out = res;
out:
    free(f);
    free(rho);
    free(ux);
    free(uy);
    free(pux);
    free(puy);
    free(uin);
    return status;
}

int orc_run(int nx, int ny, const uint8_t *type, double tau, double u_peak,
            double rho_out, double *fs, int64_t max_steps, double tol,
            int32_t check_every, int32_t collide, int64_t *steps_done,
            double *res_out) {
    return orc_run_ex(nx, ny, type, tau, u_peak, rho_out, 0, fs, max_steps, tol,
                      check_every, collide, steps_done, res_out);
}

/* Sums over the boundary columns of one stored state: per-outlet mass flux
 * (outlets are the maximal runs of outlet cells in column nx-1, ordered by y;
 * each flux is the sum over its cells of rho*u_x, the x momentum of Eq. 2,
 * taken in increasing y), the inlet flux, and the density sums and counts of
 * the inlet and outlet cells.  Returns the number of outlets, or ORC_EINVAL if
 * it exceeds cap. */
static int boundary_sums(int nx, int ny, const uint8_t *type, const double *fs, double *flow,
                         int cap, double *flow_in, double *rho_in_sum, long *cnt_in,
                         double *rho_out_sum, long *cnt_out) {
    const size_t N = (size_t)nx * ny;
    double fc[Q], r, jx, jy;
    int nout = 0, inrun = 0;
    double rin = 0.0, rout = 0.0, fin = 0.0;
    long ci = 0, co = 0;
    for (int y = 0; y < ny; ++y) {
        size_t n = (size_t)y * nx + (nx - 1);
        if (type[n] == T_OUTLET) {
            for (int i = 0; i < Q; ++i) fc[i] = fs[i * N + n];
            moments9(fc, &r, &jx, &jy);
            if (!inrun) {
                if (nout >= cap) return ORC_EINVAL;
                flow[nout++] = 0.0;
                inrun = 1;
            }
            flow[nout - 1] += jx;
            rout += r;
            ++co;
        } else {
            inrun = 0;
        }
        n = (size_t)y * nx;
        if (type[n] == T_INLET) {
            for (int i = 0; i < Q; ++i) fc[i] = fs[i * N + n];
            moments9(fc, &r, &jx, &jy);
            fin += jx;
            rin += r;
            ++ci;
        }
    }
    *flow_in = fin;
    *rho_in_sum = rin;
    *cnt_in = ci;
    *rho_out_sum = rout;
    *cnt_out = co;
    return nout;
}

/* Sum of rho over the non-solid cells, row-major. */
static double mass_sum(int nx, int ny, const uint8_t *type, const double *fs) {
    const size_t N = (size_t)nx * ny;
    double fc[Q], r, jx, jy, m = 0.0;
    for (size_t n = 0; n < N; ++n) {
        if (type[n] == T_SOLID) continue;
        for (int i = 0; i < Q; ++i) fc[i] = fs[i * N + n];
        moments9(fc, &r, &jx, &jy);
        m += r;
    }
    return m;
}

/* Pressure drop c_s^2 (mean rho over inlet cells - mean rho over outlet
 * cells), Eq. 4. */
static double pressure_drop(double rho_in_sum, long cnt_in, double rho_out_sum, long cnt_out) {
    double rin = cnt_in ? rho_in_sum / (double)cnt_in : 0.0;
    double rout = cnt_out ? rho_out_sum / (double)cnt_out : 0.0;
    return (rin - rout) / INV_CS2;
}

/* theta (Eq. 9) and D_g (Eq. 10, with mdot_ave of Eq. 11; 0 for one outlet). */
static void uniformity(const double *flow, int nout, double *theta, double *dg) {
    if (nout > 0) {
        double mx = flow[0], mn = flow[0], s = 0.0;
        for (int k = 0; k < nout; ++k) {
            if (flow[k] > mx) mx = flow[k];
            if (flow[k] < mn) mn = flow[k];
            s += flow[k];
        }
        double ave = s / (double)nout;
        *theta = mx / mn;
        double d = 0.0;
        for (int k = 0; k < nout; ++k) {
            double e = flow[k] / ave - 1.0;
            d += e * e;
        }
        *dg = nout > 1 ? sqrt(d / (double)(nout - 1)) : 0.0;
    } else {
        *theta = 0.0;
        *dg = 0.0;
    }
}

/*
 * Boundary reductions of Sec. 4.2 on one stored state.
 *   flow[k]   mass flux of outlet k (boundary_sums);
 *   flow_in   the same over the inlet cells;
 *   dp        Eq. 4; theta Eq. 9; dg Eq. 10 with Eq. 11;
 *   mass      sum of rho over non-solid cells, row-major.
 * Returns the number of outlets, or ORC_EINVAL if it exceeds cap.
 */
int orc_outlet_stats(int nx, int ny, const uint8_t *type, const double *fs,
                     double *flow, int cap, double *flow_in, double *dp,
                     double *theta, double *dg, double *mass) {
    if (check_types(nx, ny, type) != ORC_OK) return ORC_EINVAL;
    double rin, rout;
    long ci, co;
    int nout = boundary_sums(nx, ny, type, fs, flow, cap, flow_in, &rin, &ci, &rout, &co);
    if (nout < 0) return nout;
    *mass = mass_sum(nx, ny, type, fs);
    *dp = pressure_drop(rin, ci, rout, co);
    uniformity(flow, nout, theta, dg);
    return nout;
}

/*
 * The same reductions as the steady flow rates of the method: the mean over
 * the stored state and the state one time step later.
 *
 * Reading: at a converged state the boundary fluxes still carry an undamped
 * oscillation of period two time steps (a lattice mode at the Nyquist
 * frequency in time, localised at the fixed-density outlets: a few percent of
 * the outlet flux on the distributors, halving per column into the domain).
 * The residual of the steady-state test compares velocities a whole number of
 * check intervals apart and cannot see it, and rounding perturbations of that
 * mode never decay, so a flux taken at one step is not a property of the
 * steady flow.  The mean of two consecutive steps cancels the mode; it is
 * steady to round-off and satisfies the inflow/outflow balance.
 *
 *   flow[k], flow_in   means of the two states' fluxes, 0.5 * (a + b);
 *   dp                 0.5 * (dp_a + dp_b);
 *   theta, dg          Eqs. 9-11 on the mean fluxes;
 *   mass               the stored state's mass (bookkeeping, not averaged);
 *   flow_p2            largest period-two component, max_k |a_k - b_k| / 2.
 * The stored state is not modified.  Returns the number of outlets, or
 * ORC_EINVAL / ORC_ENOMEM.
 */
int orc_outlet_stats2(int nx, int ny, const uint8_t *type, double tau, double u_peak,
                      double rho_out, int32_t flags, const double *fs, double *flow, int cap,
                      double *flow_in, double *dp, double *theta, double *dg, double *mass,
                      double *flow_p2) {
    if (check_types(nx, ny, type) != ORC_OK || cap < 0) return ORC_EINVAL;
    const size_t N = (size_t)nx * ny;
    double *g = malloc(sizeof(double) * Q * N);
    double *fb = malloc(sizeof(double) * (cap > 0 ? cap : 1));
    int nout = ORC_ENOMEM;
    if (!g || !fb) goto out;
    memcpy(g, fs, sizeof(double) * Q * N);
    int64_t done = 0;
    int rc = orc_run_ex(nx, ny, type, tau, u_peak, rho_out, flags, g, 1, 0.0, 1, 1, &done, NULL);
    if (rc != ORC_OK && rc != ORC_EUNSTABLE) {
        nout = rc;
        goto out;
    }
    double fin_a, fin_b, rin_a, rin_b, rout_a, rout_b;
    long ci_a, ci_b, co_a, co_b;
    nout = boundary_sums(nx, ny, type, fs, flow, cap, &fin_a, &rin_a, &ci_a, &rout_a, &co_a);
    if (nout < 0) goto out;
    boundary_sums(nx, ny, type, g, fb, cap, &fin_b, &rin_b, &ci_b, &rout_b, &co_b);
    double p2 = 0.0;
    for (int k = 0; k < nout; ++k) {
        double h = fabs(flow[k] - fb[k]) * 0.5;
        if (h > p2) p2 = h;
        flow[k] = 0.5 * (flow[k] + fb[k]);
    }
    *flow_in = 0.5 * (fin_a + fin_b);
    *dp = 0.5 * (pressure_drop(rin_a, ci_a, rout_a, co_a) +
                 pressure_drop(rin_b, ci_b, rout_b, co_b));
    *mass = mass_sum(nx, ny, type, fs);
    *flow_p2 = p2;
    uniformity(flow, nout, theta, dg);
out:
    free(g);
    free(fb);
    return nout;
}

/* SplitMix64 (Steele, Lea & Flood, OOPSLA 2014): the first output of a
 * generator whose state is `state`, i.e. the finaliser applied to
 * state + golden gamma. */
uint64_t orc_splitmix64(uint64_t state) {
    uint64_t z = state + 0x9e3779b97f4a7c15ULL;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

/* One candidate of the exchange step. */
typedef struct {
    double key;
    uint64_t hash;
    int64_t idx;
} cand_t;

static int cmp_ascending(const void *pa, const void *pb) {
    const cand_t *a = pa, *b = pb;
    if (a->key < b->key) return -1;
    if (a->key > b->key) return 1;
    if (a->hash < b->hash) return -1;
    if (a->hash > b->hash) return 1;
    return (a->idx > b->idx) - (a->idx < b->idx);
}

static int cmp_descending(const void *pa, const void *pb) {
    const cand_t *a = pa, *b = pb;
    if (a->key > b->key) return -1;
    if (a->key < b->key) return 1;
    if (a->hash < b->hash) return -1;
    if (a->hash > b->hash) return 1;
    return (a->idx > b->idx) - (a->idx < b->idx);
}

enum { CRIT_PAPER = 0, CRIT_SPEED = 1 };
enum { REINIT_WARM = 0, REINIT_COLD = 1 };

/*
 * Exchange step of Sec. 2.2 / step (3) of Sec. 2.3 on a given field.
 *
 * Interface cells are the cells inside the eligible band
 * (band_x <= x <= nx-1-band_x, band_y <= y <= ny-1-band_y) with a 4-neighbour
 * of the other phase: fluid cells (type 1 only) touching a solid cell, and
 * solid cells touching a non-solid cell (fluid, inlet or outlet).
 *
 * Criterion PAPER:
 *   fluid key = rho |u|^2 (Eq. 6; the factor 1/2 does not change the order),
 *   evaluated as t1 = ux*ux, t2 = uy*uy, t3 = t1 + t2, key = rho*t3;
 *   solid key = sum over the non-solid 4-neighbours, in the order
 *   E(+x), N(+y), W(-x), S(-y), of the tangential speed they drag along the
 *   shared face: |u_y| across the E and W faces, |u_x| across N and S
 *   (Eq. 5 without the common factor mu/(0.5 dx)), summed left to right
 *   starting from 0.
 * Criterion SPEED: fluid key = t1 + t2; solid key = max of (t1 + t2) over the
 * non-solid 4-neighbours.
 *
 * K = max(1, floor(frac * N_f)) with N_f the number of type-1 cells;
 * K_eff = min(K, |C_f|, |C_s|).  The K_eff fluid candidates with the lowest
 * keys become solid and the K_eff solid candidates with the highest keys
 * become fluid, both chosen from the mask passed in.  Ties are broken by
 * ascending splitmix64(seed + idx), then ascending idx.
 *
 * If fs is given it is reinitialised: WARM sets the populations of new fluid
 * cells to w_i and zeroes those of new solid cells; COLD resets every
 * non-solid cell to w_i.
 *
 * removed / added (capacity `cap` each, may be NULL) receive the flipped cell
 * indices in selection order.  mass_removed sums rho over the removed cells in
 * that order; mass_added = K_eff (each new fluid cell starts at rho = 1).
 * Returns K_eff >= 0, or ORC_EINVAL on bad input (including a negative or NaN
 * key), ORC_ENOMEM.
 */
int orc_shape_update(int nx, int ny, uint8_t *type, const double *rho,
                     const double *ux, const double *uy, double frac,
                     uint64_t seed, int band_x, int band_y, int criterion,
                     int reinit, double *fs, int64_t *removed,
                     int64_t *added, int cap, double *mass_removed,
                     double *mass_added, int64_t *nf_before,
                     int64_t *nf_after) {
    if (check_types(nx, ny, type) != ORC_OK) return ORC_EINVAL;
    if (!(frac >= 0.0 && frac <= 1.0) || band_x < 1 || band_y < 1 ||
        (criterion != CRIT_PAPER && criterion != CRIT_SPEED) ||
        (reinit != REINIT_WARM && reinit != REINIT_COLD))
        return ORC_EINVAL;
    const size_t N = (size_t)nx * ny;
    int64_t nf = 0;
    for (size_t n = 0; n < N; ++n) nf += type[n] == T_FLUID;
    int64_t K = (int64_t)floor(frac * (double)nf);
    if (K < 1) K = 1;

    cand_t *cf = malloc(sizeof(cand_t) * (N ? N : 1));
    cand_t *cs = malloc(sizeof(cand_t) * (N ? N : 1));
    if (!cf || !cs) {
        free(cf);
        free(cs);
        return ORC_ENOMEM;
    }
    size_t nfc = 0, nsc = 0;
    /* neighbour order E, N, W, S */
    const int DX[4] = {1, 0, -1, 0};
    const int DY[4] = {0, 1, 0, -1};
    int bad = 0;
    for (int y = band_y; y <= ny - 1 - band_y; ++y) {
        for (int x = band_x; x <= nx - 1 - band_x; ++x) {
            size_t n = (size_t)y * nx + x;
            if (type[n] == T_FLUID) {
                int touches = 0;
                for (int d = 0; d < 4; ++d)
                    touches |= type[(size_t)(y + DY[d]) * nx + x + DX[d]] ==
                               T_SOLID;
                if (!touches) continue;
                double t1 = ux[n] * ux[n];
                double t2 = uy[n] * uy[n];
                double t3 = t1 + t2;
                double key = criterion == CRIT_PAPER ? rho[n] * t3 : t3;
                if (!(key >= 0.0)) bad = 1;
                cf[nfc].key = key;
                cf[nfc].hash = orc_splitmix64(seed + (uint64_t)n);
                cf[nfc].idx = (int64_t)n;
                ++nfc;
            } else if (type[n] == T_SOLID) {
                int touches = 0;
                double key = 0.0;
                for (int d = 0; d < 4; ++d) {
                    size_t m = (size_t)(y + DY[d]) * nx + x + DX[d];
                    if (type[m] == T_SOLID) continue;
                    touches = 1;
                    if (criterion == CRIT_PAPER) {
                        double tang = DX[d] != 0 ? fabs(uy[m]) : fabs(ux[m]);
                        key = key + tang;
                    } else {
                        double t1 = ux[m] * ux[m];
                        double t2 = uy[m] * uy[m];
                        double s = t1 + t2;
                        if (!(s >= 0.0)) bad = 1;
                        if (s > key) key = s;
                    }
                }
                if (!touches) continue;
                if (!(key >= 0.0)) bad = 1;
                cs[nsc].key = key;
                cs[nsc].hash = orc_splitmix64(seed + (uint64_t)n);
                cs[nsc].idx = (int64_t)n;
                ++nsc;
            }
        }
    }
    if (bad) {
        free(cf);
        free(cs);
        return ORC_EINVAL;
    }
    qsort(cf, nfc, sizeof(cand_t), cmp_ascending);
    qsort(cs, nsc, sizeof(cand_t), cmp_descending);
    int64_t keff = K;
    if ((int64_t)nfc < keff) keff = (int64_t)nfc;
    if ((int64_t)nsc < keff) keff = (int64_t)nsc;

    double mr = 0.0;
    for (int64_t k = 0; k < keff; ++k) mr += rho[cf[k].idx];
    for (int64_t k = 0; k < keff; ++k) {
        type[cf[k].idx] = T_SOLID;
        type[cs[k].idx] = T_FLUID;
        if (removed && k < cap) removed[k] = cf[k].idx;
        if (added && k < cap) added[k] = cs[k].idx;
    }
    if (fs) {
        if (reinit == REINIT_WARM) {
            for (int64_t k = 0; k < keff; ++k) {
                for (int i = 0; i < Q; ++i) {
                    fs[i * N + cf[k].idx] = 0.0;
                    fs[i * N + cs[k].idx] = WT[i];
                }
            }
        } else {
            for (size_t n = 0; n < N; ++n)
                for (int i = 0; i < Q; ++i)
                    fs[i * N + n] = type[n] == T_SOLID ? 0.0 : WT[i];
        }
    }
    int64_t nf2 = 0;
    for (size_t n = 0; n < N; ++n) nf2 += type[n] == T_FLUID;
    *mass_removed = mr;
    *mass_added = (double)keff * 1.0;
    *nf_before = nf;
    *nf_after = nf2;
    free(cf);
    free(cs);
    return (int)keff;
}

/* Number of OpenMP threads the per-cell passes use (1 without OpenMP). */
int orc_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Set the number of OpenMP threads of the per-cell passes (timing only: the
 * results do not depend on it). */
void orc_set_num_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
