"""Comparison helpers shared by the GPU parity tests: relative field errors
with the oracle's rounding floors, outlet statistics against the oracle's
two-step means, and the FP64 state digest computed from an oracle state."""
import math

import numpy as np

EPS = np.finfo(np.float64).eps


def field_errors(types, g_field, o_field):
    """(relative L2 error of u, of rho - 1) over non-solid cells, each divided
    by its allowance for the given precision tolerance.  The oracle forms
    rho = sum f_i with f_i = O(w_i), so its rho carries up to ~4 eps of
    absolute rounding: relative to rho - 1 that is 4 eps |rho| / |rho - 1|,
    added to the allowance (8 eps to cover both sides)."""
    ns = types != 0
    rg, xg, yg = (a[ns] for a in g_field)
    ro, xo, yo = (a[ns] for a in o_field)
    du = math.sqrt(((xg - xo) ** 2 + (yg - yo) ** 2).sum()) / \
        max(math.sqrt((xo ** 2 + yo ** 2).sum()), 1e-300)
    dnorm = max(np.linalg.norm(ro - 1.0), 1e-300)
    dr = np.linalg.norm(rg - ro) / dnorm
    floor = 8 * EPS * np.linalg.norm(ro) / dnorm
    return du, dr, floor


def fields_ok(types, g_field, o_field, tol, tag=""):
    du, dr, floor = field_errors(types, g_field, o_field)
    report(f"fields {tag}", du=du, drho=dr, drho_floor=floor)
    return du < tol and dr < tol + floor


def _outlet_l1(o):
    """Per outlet: number of cells and the sum over its cells of |rho u_x|."""
    t = o.types
    rho, ux, _ = o.macro()
    col = t[:, -1]
    counts, l1, y = [], [], 0
    while y < len(col):
        if col[y] == 3:
            y0 = y
            while y < len(col) and col[y] == 3:
                y += 1
            counts.append(y - y0)
            l1.append(float(np.abs(rho[y0:y, -1] * ux[y0:y, -1]).sum()))
        else:
            y += 1
    return np.array(counts), np.array(l1), max(1.0, float(rho.max()))


def stats_ok(g, o, tol, tag=""):
    """Outlet fluxes and the pressure drop against the oracle.  A flux is a
    sum over n cells of j_x = sum c_x f_i: its error is judged relative to the
    sum of |rho u_x| over those cells (the flux's own condition), plus the
    oracle's rounding floor of ~4 eps rho per cell; dp is a difference of
    mean densities, floor 8 eps."""
    fg, sg = g.stats()
    so = o.outlet_stats2()
    counts, l1, rho_max = _outlet_l1(o)
    allow_f = tol * l1 + 4 * EPS * counts * rho_max
    ef = float(np.max(np.abs(fg - so.flow) / allow_f)) if len(so.flow) else 0.0
    edp = abs(sg.dp - so.dp) / (tol * abs(so.dp) + 8 * EPS * rho_max)
    report(f"stats {tag}", flux_over_allow=ef, dp_over_allow=edp,
           flux_rel=float(np.max(np.abs(fg - so.flow) / np.abs(so.flow))) if len(so.flow) else 0.0,
           dp_rel=abs(sg.dp - so.dp) / abs(so.dp) if so.dp else 0.0)
    return ef < 1.0 and edp < 1.0, sg, so


def report(tag, **kw):
    print(tag, " ".join(f"{k}={v:.3e}" if isinstance(v, float) else f"{k}={v}"
                        for k, v in kw.items()), flush=True)


_GAMMA = np.uint64(0x9E3779B97F4A7C15)


def _splitmix64(s):
    """SplitMix64 output function on s + gamma (Steele, Lea & Flood 2014),
    elementwise on uint64 arrays (arithmetic mod 2^64)."""
    with np.errstate(over="ignore"):
        z = s + _GAMMA
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        return z ^ (z >> np.uint64(31))


def f64_state_digest(types, fs):
    """The library's order-free state digest (sum mod 2^64 over cells of
    SplitMix64 of each stored population's bits mixed with its position,
    plus each cell's type) for a double-precision state given as the oracle
    holds it: fs (9, ny, nx) float64, types (ny, nx)."""
    t = np.ascontiguousarray(types, np.uint8).ravel().astype(np.uint64)
    n = np.arange(t.size, dtype=np.uint64)
    with np.errstate(over="ignore"):
        acc = _splitmix64(t ^ (n << np.uint64(8)) ^ np.uint64(0xD1B54A32D192ED03)).sum(
            dtype=np.uint64)
        live = t != 0
        bits = np.ascontiguousarray(fs, np.float64).reshape(9, -1).view(np.uint64)
        for i in range(9):
            pos = (np.uint64(9) * n[live] + np.uint64(i)) * _GAMMA
            acc += _splitmix64(bits[i][live] ^ pos).sum(dtype=np.uint64)
    return int(acc)
