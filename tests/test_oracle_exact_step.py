"""Brute-force pin of one whole time step of the oracle, in exact arithmetic.

An 8 x 8 lattice with all four cell types (an inlet opening and two outlet
openings with their end cells, an obstacle, and a solid cell in a wall
corner) is advanced one step with Python fractions, then compared with the
oracle's FP64 step.  The exact step is written independently of the oracle:

* streaming in push form (each population leaves its cell along c_i and either
  lands on the neighbour or, at a wall, comes back reversed), Eq. 1;
* the inlet and outlet closures solved as linear systems from their defining
  conditions (imposed velocity or density, zero transverse momentum, and
  bounce-back of the non-equilibrium part of the population normal to the
  boundary) instead of the closed-form expressions;
* the equilibrium in its tensor form w_i rho [1 + c.u/cs^2 + Q_i:uu/(2 cs^4)],
  Q_i = c_i c_i - cs^2 I (the second-order equilibrium of Sec. 2.1);
* the relaxation of Eq. 1 with 1/tau, tau = 4/5 (so omega = 5/4 differs from
  tau, and tau = 1 is avoided).

Inputs are doubles, converted exactly; the inlet parabola's parameters are
chosen so that the imposed velocities are exact binary fractions.  The oracle
must agree with the exact result to round-off: along any population's
dependency chain a double step rounds a few tens of times (a closure about
eight operations, the 9-term moment sums, the division by rho, the equilibrium
polynomial, the relaxation), each contributing at most half an ulp scaled by
a coefficient of order one, so every population must lie within 16 ulp of the
exact value and the mean error within 2 ulp (measured: at most 10 ulp, mean
1.2-1.5 ulp over six seeds; the worst cases are inlet and outlet cells).  A
wrong coefficient, sign or index moves a population by more than 1e-4
relative, some 10^11 ulp.
"""
import math
from fractions import Fraction as Fr

import numpy as np
import pytest

SOLID, FLUID, INLET, OUTLET = 0, 1, 2, 3


def paper_velocity_set():
    """c_i from the angles of Sec. 2.1 (diagonals at 45 + (i-5) 90 degrees,
    length sqrt 2), and the weights 4/9, 1/9, 1/36."""
    c = [(0, 0)]
    for i in range(1, 5):
        a = (i - 1) * math.pi / 2
        c.append((round(math.cos(a)), round(math.sin(a))))
    for i in range(5, 9):
        a = (i - 5) * math.pi / 2 + math.pi / 4
        c.append((round(math.sqrt(2) * math.cos(a)), round(math.sqrt(2) * math.sin(a))))
    w = [Fr(4, 9)] + [Fr(1, 9)] * 4 + [Fr(1, 36)] * 4
    opp = [c.index((-cx, -cy)) for cx, cy in c]
    return c, w, opp


C, W, OPP = paper_velocity_set()
CS2 = Fr(1, 3)


def feq_exact(rho, ux, uy):
    out = []
    for (cx, cy), w in zip(C, W):
        cu = cx * ux + cy * uy
        quu = (cx * cx - CS2) * ux * ux + 2 * cx * cy * ux * uy + (cy * cy - CS2) * uy * uy
        out.append(w * rho * (1 + cu / CS2 + quu / (2 * CS2 * CS2)))
    return out


def solve(a, b):
    """Exact Gaussian elimination for a small square system a x = b."""
    n = len(b)
    m = [list(r) + [v] for r, v in zip(a, b)]
    for col in range(n):
        piv = next(r for r in range(col, n) if m[r][col] != 0)
        m[col], m[piv] = m[piv], m[col]
        for r in range(n):
            if r != col and m[r][col] != 0:
                k = m[r][col] / m[col][col]
                m[r] = [x - k * y for x, y in zip(m[r], m[col])]
    return [m[i][n] / m[i][i] for i in range(n)]


def lattice_8x8():
    t = np.full((8, 8), FLUID, np.uint8)
    t[0, :] = SOLID
    t[7, :] = SOLID
    t[:, 0] = SOLID
    t[2:6, 0] = INLET          # opening rows 2..5: both end cells touch walls
    t[:, 7] = SOLID
    t[1:3, 7] = OUTLET         # outlet touching the bottom wall (a corner)
    t[4:7, 7] = OUTLET         # second outlet touching the top wall
    t[3:5, 3] = SOLID          # obstacle
    t[1, 5] = SOLID            # solid cell in the bottom-wall corner
    return t


def inlet_velocity(t, u_peak):
    """Parabola of Sec. 3.3 over the inlet run, walls half a cell outside."""
    rows = [y for y in range(t.shape[0]) if t[y, 0] == INLET]
    y0, y1 = rows[0], rows[-1]
    wdt = y1 - y0 + 1
    return {y: 4 * u_peak * (y - y0 + Fr(1, 2)) * (y1 + Fr(1, 2) - y) / (wdt * wdt)
            for y in rows}


def exact_step(t, fs, tau, u_peak, rho_out):
    ny, nx = t.shape
    live = lambda x, y: 0 <= x < nx and 0 <= y < ny and t[y, x] != SOLID
    f = {}
    # push streaming with halfway bounce-back
    for y in range(ny):
        for x in range(nx):
            if t[y, x] == SOLID:
                continue
            for i, (cx, cy) in enumerate(C):
                if live(x + cx, y + cy):
                    f[(x + cx, y + cy, i)] = fs[i][y][x]
                else:
                    f[(x, y, OPP[i])] = fs[i][y][x]
    # the odd part of feq_i - feq_opp(i) at unit density along x (linear in u_x)
    d13 = (feq_exact(1, 1, 0)[1] - feq_exact(1, 1, 0)[3]
           - feq_exact(1, -1, 0)[1] + feq_exact(1, -1, 0)[3]) / 2
    uin = inlet_velocity(t, u_peak)
    for y in range(ny):
        if t[y, 0] == INLET:
            g = [f[(0, y, i)] for i in range(9)]
            ux = uin[y]
            # unknowns f1, f5, f8, rho: mass, x momentum, zero y momentum,
            # and f1 - f3 = feq1 - feq3 = rho d13 ux
            a = [[1, 1, 1, -1], [1, 1, 1, -ux], [0, 1, -1, 0], [1, 0, 0, -d13 * ux]]
            b = [-(g[0] + g[2] + g[3] + g[4] + g[6] + g[7]), g[3] + g[6] + g[7],
                 -(g[2] + g[6] - g[4] - g[7]), g[3]]
            f1, f5, f8, _ = solve(a, b)
            f[(0, y, 1)], f[(0, y, 5)], f[(0, y, 8)] = f1, f5, f8
        x = nx - 1
        if t[y, x] == OUTLET:
            g = [f[(x, y, i)] for i in range(9)]
            # unknowns f3, f6, f7, u_x at density rho_out with zero y momentum,
            # and f3 - f1 = feq3 - feq1 = -rho_out d13 u_x
            a = [[1, 1, 1, 0], [-1, -1, -1, -rho_out], [0, 1, -1, 0], [1, 0, 0, rho_out * d13]]
            b = [rho_out - (g[0] + g[1] + g[2] + g[4] + g[5] + g[8]), -(g[1] + g[5] + g[8]),
                 -(g[2] + g[5] - g[4] - g[8]), g[1]]
            f3, f6, f7, _ = solve(a, b)
            f[(x, y, 3)], f[(x, y, 6)], f[(x, y, 7)] = f3, f6, f7
    out = [[[Fr(0)] * nx for _ in range(ny)] for _ in range(9)]
    for y in range(ny):
        for x in range(nx):
            if t[y, x] == SOLID:
                continue
            g = [f[(x, y, i)] for i in range(9)]
            rho = sum(g)
            ux = sum(gi * c[0] for gi, c in zip(g, C)) / rho
            uy = sum(gi * c[1] for gi, c in zip(g, C)) / rho
            eq = feq_exact(rho, ux, uy)
            for i in range(9):
                out[i][y][x] = g[i] - (g[i] - eq[i]) / tau
    return out


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_one_step_matches_exact_arithmetic(orc, seed):
    t = lattice_8x8()
    ny, nx = t.shape
    rng = np.random.default_rng(seed)
    w = np.array([float(x) for x in W])
    fs = w[:, None, None] * (1 + 0.1 * rng.uniform(-1, 1, (9, ny, nx)))
    fs[:, t == SOLID] = 0.0
    tau_exact, u_peak, rho_out = Fr(4, 5), 0.0625, 1.0
    lat = orc.Lattice(t, 0.8, u_peak, rho_out)
    lat.fs[:] = fs
    status, steps, _ = lat.run(1, 0.0, 1)
    assert status == orc.OK and steps == 1
    exact = exact_step(t, [[[Fr(float(v)) for v in row] for row in plane] for plane in fs],
                       tau_exact, Fr(u_peak), Fr(rho_out))
    errs = []
    for i in range(9):
        for y in range(ny):
            for x in range(nx):
                if t[y, x] == SOLID:
                    assert lat.fs[i, y, x] == 0.0
                    continue
                e = float(exact[i][y][x])
                errs.append(abs(lat.fs[i, y, x] - e) / math.ulp(abs(e)))
    errs = np.array(errs)
    assert errs.max() <= 16.0, f"oracle step differs from exact arithmetic by {errs.max():.1f} ulp"
    assert errs.mean() <= 2.0, f"mean error {errs.mean():.2f} ulp"


def test_exact_step_distinguishes_the_relaxation_rate(orc):
    """The exact step is sensitive to the relaxation rate: relaxing with omega
    = tau instead of 1/tau moves the result by far more than the tolerance."""
    t = lattice_8x8()
    ny, nx = t.shape
    rng = np.random.default_rng(5)
    w = np.array([float(x) for x in W])
    fs = w[:, None, None] * (1 + 0.1 * rng.uniform(-1, 1, (9, ny, nx)))
    fs[:, t == SOLID] = 0.0
    ex = [[[Fr(float(v)) for v in row] for row in plane] for plane in fs]
    right = exact_step(t, ex, Fr(4, 5), Fr(0.0625), Fr(1))
    wrong = exact_step(t, ex, Fr(5, 4), Fr(0.0625), Fr(1))
    diff = max(abs(float(right[i][y][x] - wrong[i][y][x]))
               for i in range(9) for y in range(ny) for x in range(nx))
    assert diff > 1e-4
