"""Seeded synthetic inputs: cell-type maps and random population states.

This module holds no lattice-Boltzmann arithmetic.  It builds the workloads
both the GPU library and the CPU oracle are run on, and nothing else; it
imports neither of them.

Cell types follow Sec. 3.3 / Fig. 5: 0 solid, 1 fluid, 2 inlet, 3 outlet.
Inlet cells are the open cells of column 0, outlet cells the open cells of
column nx-1.

The paper's own distributor drawing (Fig. 4/5) is not available, so the
distributor is a flat binary tree built from the description of Sec. 3.2 (an
inlet channel that splits by successive T bifurcations into 2^L equally spaced
outlets, channel widths shrinking per generation) at lattice resolution:

  * branch centres yc(k, j) = floor((2j+1) ny / 2^(k+1)), k = 0..L, j < 2^k;
  * junction columns xj(k) = round((k+1) nx / (L+1));
  * the level-k bars, w_k rows wide, run from xj(k-1) (0 for k = 0) to xj(k)
    (nx for k = L) on rows [yc - floor(w_k/2), yc - floor(w_k/2) + w_k);
  * at xj(k) a connector w_{k+1} columns wide joins children 2j and 2j+1;
  * rows 0 and ny-1 and every cell not in a bar or connector are solid.
"""
from __future__ import annotations

import dataclasses
import math
from dataclasses import dataclass, field

import numpy as np

SOLID, FLUID, INLET, OUTLET = 0, 1, 2, 3


def _mark_ports(t: np.ndarray) -> np.ndarray:
    nx = t.shape[1]
    t[0, :] = SOLID
    t[-1, :] = SOLID
    col0 = t[:, 0] != SOLID
    t[col0, 0] = INLET
    coln = t[:, nx - 1] != SOLID
    t[coln, nx - 1] = OUTLET
    return t


def default_widths(ny: int, levels: int) -> list[int]:
    """w_0 = ny/8 halving per generation (the 1024x512 and 2048x1024
    distributors), floored at 2."""
    return [max(2, (ny // 8) >> k) for k in range(levels + 1)]


def check_widths(ny: int, levels: int, widths) -> None:
    if levels < 1 or levels > 8:
        raise ValueError("levels must be in 1..8")
    if len(widths) != levels + 1:
        raise ValueError("need levels+1 widths")
    if min(widths) < 2:
        raise ValueError("widths must be >= 2")
    if ny // (2 ** levels) < widths[levels] + 2:
        raise ValueError("outlet channels do not fit: ny/2^L < w_L + 2")


def distributor(nx: int, ny: int, levels: int, widths=None) -> np.ndarray:
    """Flat arborescent distributor with one inlet and 2^levels outlets."""
    widths = list(widths) if widths is not None else default_widths(ny, levels)
    check_widths(ny, levels, widths)
    L = levels
    t = np.zeros((ny, nx), np.uint8)
    xj = [int(round((k + 1) * nx / (L + 1))) for k in range(L)] + [nx]

    def yc(k, j):
        return ((2 * j + 1) * ny) // (2 ** (k + 1))

    for k in range(L + 1):
        w = widths[k]
        xs = 0 if k == 0 else xj[k - 1]
        xe = xj[k]
        for j in range(2 ** k):
            r0 = yc(k, j) - w // 2
            t[max(r0, 0):min(r0 + w, ny), xs:xe] = FLUID
        if k < L:
            wc = widths[k + 1]
            c0 = xj[k] - wc // 2
            for j in range(2 ** k):
                ya = yc(k + 1, 2 * j) - wc // 2
                yb = yc(k + 1, 2 * j + 1) - wc // 2 + wc
                t[max(ya, 0):min(yb, ny), max(c0, 0):min(c0 + wc, nx)] = FLUID
    return _mark_ports(t)


def collector(nx: int, ny: int, levels: int, widths=None) -> np.ndarray:
    """The flow direction of the paper's own run (Sec. 3.3): the distributor's
    channels mirrored left to right, so 2^levels inlets on column 0 (the
    former outlets, equal widths, hence equal parabolic flow rates) merge into
    one outlet on column nx-1."""
    t = distributor(nx, ny, levels, widths)
    fluid = (t != SOLID)[:, ::-1]
    out = np.where(fluid, FLUID, SOLID).astype(np.uint8)
    return _mark_ports(out)


def t_junction(nx: int, ny: int, w_in: int, w_out: int) -> np.ndarray:
    """Synthetic T-junction (the elemental example of Sec. 2.3, whose figure
    is not available): an inlet stem w_in rows wide along the mid-height meets
    a crossbar w_out columns wide at x = nx/2 at right angles; two arms w_out
    rows wide leave its ends at y = ny/4 and 3ny/4 for the outlets on column
    nx-1.  It is the one-level tree of the distributor generator."""
    return distributor(nx, ny, 1, [w_in, w_out])


def lower_half(types: np.ndarray) -> np.ndarray:
    """Rows 0..ny/2-1 of a map that is mirror symmetric about the line
    between rows ny/2-1 and ny/2 (checked): the computational domain of a
    half-domain run with a symmetry plane above its top row (Sec. 3.3)."""
    ny = types.shape[0]
    if ny % 2 or not np.array_equal(types, types[::-1]):
        raise ValueError("map is not mirror symmetric about its mid line")
    return np.ascontiguousarray(types[: ny // 2])


def channel(nx: int, ny: int) -> np.ndarray:
    """Straight channel: solid rows 0 and ny-1, inlet column 0, outlet column
    nx-1, fluid elsewhere (the all-fluid throughput workload and the
    Poiseuille case)."""
    t = np.full((ny, nx), FLUID, np.uint8)
    return _mark_ports(t)


def closed_box(nx: int, ny: int, obstacles: int = 0, seed: int = 0) -> np.ndarray:
    """Fluid box with a solid frame and optional random solid cells; no
    inlets or outlets."""
    t = np.full((ny, nx), FLUID, np.uint8)
    t[0, :] = t[-1, :] = SOLID
    t[:, 0] = t[:, -1] = SOLID
    if obstacles:
        rng = np.random.default_rng(seed)
        ys = rng.integers(1, ny - 1, obstacles)
        xs = rng.integers(1, nx - 1, obstacles)
        t[ys, xs] = SOLID
    return t


def random_state(types: np.ndarray, seed: int, weights, amp: float = 1e-2) -> np.ndarray:
    """Random positive populations (9, ny, nx): weights[i] (1 + amp U(-1, 1))
    on non-solid cells, zero on solid cells.  The caller passes the weights;
    this module holds no lattice constant of its own."""
    rng = np.random.default_rng(seed)
    ny, nx = types.shape
    w = np.asarray(weights, np.float64).reshape(9, 1, 1)
    f = w * (1.0 + amp * rng.uniform(-1.0, 1.0, (9, ny, nx)))
    f[:, types == SOLID] = 0.0
    return f


def random_field(types: np.ndarray, seed: int, umax: float = 0.05):
    """Random (rho, ux, uy) on non-solid cells, zeros on solid cells."""
    rng = np.random.default_rng(seed)
    ny, nx = types.shape
    rho = 1.0 + 1e-3 * rng.uniform(-1, 1, (ny, nx))
    ux = umax * rng.uniform(-1, 1, (ny, nx))
    uy = umax * rng.uniform(-1, 1, (ny, nx))
    s = types == SOLID
    rho[s] = 0.0
    ux[s] = 0.0
    uy[s] = 0.0
    return rho, ux, uy


def width_law_ratio(h: float, w_next: float, tol: float = 1e-12) -> float:
    """Solve the channel-width scaling law of Sec. 3.2 (Eq. 8) for w_k given
    w_{k+1} and channel depth h, by bisection:
        (w_{k+1}/w_k)^4 (h + w_k)(3h + w_k) / ((h + w_{k+1})(3h + w_{k+1})) = 1/4.
    """
    def g(wk):
        return (w_next / wk) ** 4 * (h + wk) * (3 * h + wk) / ((h + w_next) * (3 * h + w_next)) - 0.25

    lo, hi = w_next, w_next * 4.0
    while g(hi) > 0:
        hi *= 2.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if g(mid) > 0:
            lo = mid
        else:
            hi = mid
        if hi - lo < tol * hi:
            break
    return 0.5 * (lo + hi)


def width_law_chain(h: float, w_last: float, levels: int) -> list[float]:
    """Widths w_0..w_L from the finest w_L upwards by Eq. 8."""
    ws = [w_last]
    for _ in range(levels):
        ws.append(width_law_ratio(h, ws[-1]))
    return ws[::-1]


@dataclass
class Workload:
    name: str
    nx: int
    ny: int
    levels: int
    widths: list
    tau: float
    u_peak: float
    rho_out: float = 1.0
    seed: int = 0
    kind: str = "distributor"
    extra: dict = field(default_factory=dict)

    def types(self) -> np.ndarray:
        if self.kind == "channel":
            return channel(self.nx, self.ny)
        if self.kind == "collector-half":
            return lower_half(collector(self.nx, 2 * self.ny, self.levels, self.widths))
        return distributor(self.nx, self.ny, self.levels, self.widths)


def mirror_widths(widths, ny: int) -> list[int]:
    """Round widths[k] to the nearest integer of the parity that keeps the
    generator's level-k bars mirror symmetric about the mid line of ny rows:
    even where ny / 2^(k+1) is an integer (the bar centre sits on a row
    boundary), odd otherwise (ties go to the smaller width)."""
    out = []
    for k, w in enumerate(widths):
        even = (ny % 2 ** (k + 1)) == 0
        lo = math.floor(w)
        if (lo % 2 == 0) != even:
            lo -= 1
        out.append(lo if w - lo <= lo + 2 - w else lo + 2)
    return out


def paper_collector_widths(w_in: int = 11, levels: int = 4, ny_full: int = 360) -> list[int]:
    """Channel widths in cells of the paper's own run (Sec. 3.3): the Eq. 8
    chain of Table 1 (depth 10 mm, finest channel 2 mm) scaled so that the
    finest channel is W_in cells (depth 55 cells); the trunk comes out at
    52.4 cells, the W_out of Sec. 3.3.  Rounded by mirror_widths."""
    h = 10.0 * w_in / 2.0
    return mirror_widths(width_law_chain(h, float(w_in), levels), ny_full)


# The workloads the method is exercised on (names describe them).
CORRECTNESS_128x64 = Workload("distributor-128x64-L2", 128, 64, 2, [8, 6, 4], 0.8, 0.05, seed=1,
                              extra={"warm_steps": 5000, "iters": 10, "steps_per_iter": 5000,
                                     "frac": 0.01})
HEADLINE_1024x512 = Workload("distributor-1024x512-L3", 1024, 512, 3, [64, 32, 16, 8], 0.6, 0.04,
                             seed=2, extra={"tol": 1e-6, "check_every": 100, "cap0": 500000,
                                            "iters": 50, "cap_iter": 200000, "frac": 0.01})
CHANNEL_1024x512 = Workload("channel-1024x512", 1024, 512, 0, [], 0.6, 0.04, seed=2, kind="channel")
PRECISION_2048x1024 = Workload("distributor-2048x1024-L4", 2048, 1024, 4, [128, 64, 32, 16, 8],
                               0.55, 0.03, seed=3, extra={"steps": 20000})
CHANNEL_4096x2048 = Workload("channel-4096x2048", 4096, 2048, 0, [], 0.6, 0.04, seed=2,
                             kind="channel")
# The paper's own run (Sec. 3.3): a collector computed on half its domain,
# 360 x 180 cells (the mirrored full domain 360 x 360, the square footprint of
# Sec. 3.2's outlets), 2^4 inlets of W_in = 11 cells (8 in the half), one
# outlet of W_out = 52 (26 rows in the half, against the symmetry line),
# Neumann outlet, nu = 0.04 (tau = 3 nu + 1/2 = 0.62), mean inlet velocity
# u_in = 0.08 (a parabola of peak 3/2 u_in), Re_in = 22.
PAPER_COLLECTOR_360x180 = Workload(
    "collector-half-360x180", 360, 180, 4, [52, 34, 24, 15, 11], 0.62, 0.12, seed=6,
    kind="collector-half",
    extra={"flags": 3, "nu": 0.04, "u_in": 0.08, "w_in": 11, "w_out": 52})


def batch_candidates(count: int = 256, seed: int = 4):
    """Uneven distributor candidates: nx on {128..1024} step 64, ny on
    {64..512} step 64, L in {2,3,4} (redrawn when the widths do not fit),
    w_k = max(2, round(ny/8 2^-k U(0.75, 1.25))), tau ~ U[0.55, 1.0],
    u_peak ~ U[0.02, 0.06]."""
    rng = np.random.default_rng(seed)
    out = []
    while len(out) < count:
        nx = int(rng.integers(2, 17)) * 64
        ny = int(rng.integers(1, 9)) * 64
        L = int(rng.integers(2, 5))
        ws = [max(2, int(round(ny / 8 * 2.0 ** (-k) * rng.uniform(0.75, 1.25))))
              for k in range(L + 1)]
        tau = float(rng.uniform(0.55, 1.0))
        up = float(rng.uniform(0.02, 0.06))
        try:
            check_widths(ny, L, ws)
        except ValueError:
            continue
        out.append(Workload(f"cand{len(out)}", nx, ny, L, ws, tau, up, seed=seed))
    return out


@dataclasses.dataclass
class ServeRequest:
    """One request of the serving workload: arrival time (s), lattice, storage
    form ("f32" or "f16"), kind ("solve" or "optimize") and step counts."""
    t: float
    workload: Workload
    storage: str
    kind: str
    solve_steps: int
    iterations: int
    steps_per_iteration: int
    seed: int


def serving_requests(rate: float = 50.0, seconds: float = 60.0, seed: int = 5,
                     solve_steps: int = 500, opt_warm: int = 100, opt_iters: int = 20,
                     opt_steps: int = 40):
    """Poisson arrivals (rate per second) over `seconds`.  Lattices:
    nx = 64 round(256 2^U(0,4) / 64) (256..4096), ny = nx/2; levels, widths,
    tau and u_peak drawn as in batch_candidates.  Storage FP32 / FP16 offsets
    and solve / optimize each with probability 1/2.  solve: solve_steps steps
    from rest; optimize: opt_warm steps, then opt_iters x (exchange step +
    opt_steps steps)."""
    rng = np.random.default_rng(seed)
    out = []
    t = 0.0
    while True:
        t += float(rng.exponential(1.0 / rate))
        if t >= seconds:
            break
        while True:
            nx = int(64 * round(256 * 2.0 ** rng.uniform(0.0, 4.0) / 64))
            ny = nx // 2
            L = int(rng.integers(2, 5))
            ws = [max(2, int(round(ny / 8 * 2.0 ** (-k) * rng.uniform(0.75, 1.25))))
                  for k in range(L + 1)]
            tau = float(rng.uniform(0.55, 1.0))
            up = float(rng.uniform(0.02, 0.06))
            try:
                check_widths(ny, L, ws)
                break
            except ValueError:
                continue
        storage = "f32" if rng.random() < 0.5 else "f16"
        kind = "solve" if rng.random() < 0.5 else "optimize"
        w = Workload(f"req{len(out)}", nx, ny, L, ws, tau, up, seed=seed)
        if kind == "solve":
            out.append(ServeRequest(t, w, storage, kind, solve_steps, 0, 0, len(out)))
        else:
            out.append(ServeRequest(t, w, storage, kind, opt_warm, opt_iters, opt_steps,
                                    len(out)))
    return out


def reynolds_inlet(width: float, u_in: float, nu: float) -> float:
    """Re_in = W_in u_in / nu (Sec. 3.3)."""
    return width * u_in / nu


def lattice_cells(types: np.ndarray) -> tuple[int, int]:
    """(all cells, non-solid cells)."""
    return int(types.size), int(np.count_nonzero(types != SOLID))


def log2i(n: int) -> int:
    return int(math.log2(n))
