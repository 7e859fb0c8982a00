"""FP64 CPU oracle for the LBM shape-optimisation method (Wang, Fan & Luo).

TEST INFRASTRUCTURE ONLY.  The arithmetic lives in ``lbm_oracle.c`` (plain C,
sequential reductions, no FMA contraction); this module only marshals numpy
arrays into it.  Only the tests, the smoke check and the CPU-baseline leg of
the benchmark may import it.  It imports nothing from the GPU package and the
GPU package never imports it.

Function map (paper passages):
  equilibrium, collide_cell ... Sec. 2.1, Eq. 1 and the equilibrium below it
  run_to_steady ............... Sec. 2.3 steps (2)/(4) (one LBM solve)
  residual .................... Sec. 2.3 step (2) (the steady-state test)
  macro ....................... Eq. 2
  outlet_stats ................ Eq. 4, Eqs. 9-11 on one stored state
  outlet_stats2 ............... the same as steady flow rates: mean over two
                                consecutive steps (the boundary fluxes carry an
                                undamped period-two lattice oscillation)
  shape_update ................ Sec. 2.2 (Eqs. 5, 6), Sec. 2.3 step (3)
  tau_from_nu ................. Sec. 2.1 (tau = 3 nu + dt/2)
  flags NEUMANN_OUTLET, SYMMETRY_TOP ... Sec. 3.3 (the paper's own runs:
                                zero-gradient outlet, half domain)
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lbm_oracle.c")
_LIB = os.path.join(_HERE, "liblbm_oracle.so")

OK, NOT_CONVERGED, EINVAL, ENOMEM, EUNSTABLE = 0, 1, -1, -2, -4
SOLID, FLUID, INLET, OUTLET = 0, 1, 2, 3
CRIT_PAPER, CRIT_SPEED = 0, 1
WARM, COLD = 0, 1
NEUMANN_OUTLET, SYMMETRY_TOP = 1, 2


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, no FMA contraction, OpenMP)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math",
               "-fopenmp", "-shared", "-fPIC", "-Wall", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        i32, i64, f64, u64 = ctypes.c_int, ctypes.c_int64, ctypes.c_double, ctypes.c_uint64
        lib.orc_velocity_set.argtypes = [P, P, P, P]
        lib.orc_equilibrium.argtypes = [f64, f64, f64, P]
        lib.orc_collide_cell.argtypes = [P, f64, P]
        lib.orc_tau_from_nu.argtypes = [f64]
        lib.orc_tau_from_nu.restype = f64
        lib.orc_inlet_profile.argtypes = [i32, i32, P, f64, P]
        lib.orc_inlet_profile_ex.argtypes = [i32, i32, P, f64, ctypes.c_int32, P]
        lib.orc_macro.argtypes = [i32, i32, P, P, P, P, P]
        lib.orc_init.argtypes = [i32, i32, P, P]
        lib.orc_run.argtypes = [i32, i32, P, f64, f64, f64, P, i64, f64, ctypes.c_int32,
                                ctypes.c_int32, P, P]
        lib.orc_run_ex.argtypes = [i32, i32, P, f64, f64, f64, ctypes.c_int32, P, i64, f64,
                                   ctypes.c_int32, ctypes.c_int32, P, P]
        lib.orc_outlet_stats.argtypes = [i32, i32, P, P, P, i32, P, P, P, P, P]
        lib.orc_outlet_stats2.argtypes = [i32, i32, P, f64, f64, f64, ctypes.c_int32, P, P,
                                          i32, P, P, P, P, P, P]
        lib.orc_splitmix64.argtypes = [u64]
        lib.orc_splitmix64.restype = u64
        lib.orc_shape_update.argtypes = [i32, i32, P, P, P, P, f64, u64, i32, i32, i32, i32,
                                         P, P, P, i32, P, P, P, P]
        lib.orc_num_threads.restype = i32
        lib.orc_set_num_threads.argtypes = [i32]
        lib.orc_residual.argtypes = [i32, i32, P, P, P, P, P]
        lib.orc_residual.restype = f64
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def velocity_set():
    """(cx, cy, opp, w) of the D2Q9 lattice, Sec. 2.1."""
    lib = _load()
    cx = np.zeros(9, np.int32)
    cy = np.zeros(9, np.int32)
    opp = np.zeros(9, np.int32)
    w = np.zeros(9, np.float64)
    lib.orc_velocity_set(_ptr(cx), _ptr(cy), _ptr(opp), _ptr(w))
    return cx, cy, opp, w


def equilibrium(rho: float, ux: float, uy: float) -> np.ndarray:
    out = np.zeros(9, np.float64)
    _load().orc_equilibrium(float(rho), float(ux), float(uy), _ptr(out))
    return out


def collide_cell(f, tau: float) -> np.ndarray:
    f = np.ascontiguousarray(f, np.float64)
    out = np.zeros(9, np.float64)
    _load().orc_collide_cell(_ptr(f), float(tau), _ptr(out))
    return out


def tau_from_nu(nu: float) -> float:
    return _load().orc_tau_from_nu(float(nu))


def splitmix64(state: int) -> int:
    return int(_load().orc_splitmix64(ctypes.c_uint64(state & (2**64 - 1))))


def num_threads() -> int:
    return int(_load().orc_num_threads())


def set_num_threads(n: int) -> None:
    """Threads of the per-cell passes (results do not depend on it)."""
    _load().orc_set_num_threads(int(n))


def residual(types: np.ndarray, ux, uy, ux_prev, uy_prev) -> float:
    """r = ||u - u_prev|| / ||u|| over the non-solid cells (Sec. 2.3 step 2)."""
    t = np.ascontiguousarray(types, np.uint8)
    ny, nx = t.shape
    a = [np.ascontiguousarray(v, np.float64) for v in (ux, uy, ux_prev, uy_prev)]
    for v in a:
        if v.shape != t.shape:
            raise ValueError("fields must have the shape of the type map")
    return float(_load().orc_residual(nx, ny, _ptr(t), *(_ptr(v) for v in a)))


def inlet_profile(types: np.ndarray, u_peak: float, flags: int = 0) -> np.ndarray:
    t = np.ascontiguousarray(types, np.uint8)
    ny, nx = t.shape
    out = np.zeros(ny, np.float64)
    _load().orc_inlet_profile_ex(nx, ny, _ptr(t), float(u_peak), int(flags), _ptr(out))
    return out


@dataclass
class Stats:
    flow: np.ndarray
    flow_in: float
    dp: float
    theta: float
    dg: float
    mass: float


@dataclass
class Stats2(Stats):
    flow_p2: float


@dataclass
class ShapeResult:
    k_eff: int
    removed: np.ndarray
    added: np.ndarray
    mass_removed: float
    mass_added: float
    n_fluid_before: int
    n_fluid_after: int


class Lattice:
    """One lattice: cell types (ny, nx) uint8 and the post-collision state
    fs (9, ny, nx) float64."""

    def __init__(self, types: np.ndarray, tau: float, u_peak: float, rho_out: float = 1.0,
                 flags: int = 0):
        self.types = np.ascontiguousarray(types, np.uint8).copy()
        self.ny, self.nx = self.types.shape
        self.tau, self.u_peak, self.rho_out = float(tau), float(u_peak), float(rho_out)
        self.flags = int(flags)
        self.fs = np.zeros((9, self.ny, self.nx), np.float64)
        rc = _load().orc_init(self.nx, self.ny, _ptr(self.types), _ptr(self.fs))
        if rc != OK:
            raise ValueError(f"oracle: invalid cell-type map (rc={rc})")
        self.residual = float("nan")

    def run(self, max_steps: int, tol: float = 0.0, check_every: int = 100, collide: bool = True):
        """Returns (status, steps_done, residual)."""
        steps = ctypes.c_int64(0)
        res = ctypes.c_double(0.0)
        rc = _load().orc_run_ex(self.nx, self.ny, _ptr(self.types), self.tau, self.u_peak,
                                self.rho_out, self.flags, _ptr(self.fs), int(max_steps),
                                float(tol), int(check_every), int(bool(collide)),
                                ctypes.byref(steps), ctypes.byref(res))
        if rc in (EINVAL, ENOMEM):
            raise ValueError(f"oracle run failed (rc={rc})")
        self.residual = res.value
        return rc, steps.value, res.value

    def macro(self):
        rho = np.zeros((self.ny, self.nx))
        ux = np.zeros((self.ny, self.nx))
        uy = np.zeros((self.ny, self.nx))
        rc = _load().orc_macro(self.nx, self.ny, _ptr(self.types), _ptr(self.fs), _ptr(rho),
                               _ptr(ux), _ptr(uy))
        assert rc == OK
        return rho, ux, uy

    def outlet_stats(self, cap: int = 4096) -> Stats:
        flow = np.zeros(cap)
        fin, dp, th, dg, m = (ctypes.c_double() for _ in range(5))
        n = _load().orc_outlet_stats(self.nx, self.ny, _ptr(self.types), _ptr(self.fs),
                                     _ptr(flow), cap, ctypes.byref(fin), ctypes.byref(dp),
                                     ctypes.byref(th), ctypes.byref(dg), ctypes.byref(m))
        if n < 0:
            raise ValueError(f"oracle outlet_stats failed (rc={n})")
        return Stats(flow[:n].copy(), fin.value, dp.value, th.value, dg.value, m.value)

    def outlet_stats2(self, cap: int = 4096) -> Stats2:
        """Statistics of the steady flow: the mean over this state and the
        state one step later (the state is not changed)."""
        flow = np.zeros(cap)
        fin, dp, th, dg, m, p2 = (ctypes.c_double() for _ in range(6))
        n = _load().orc_outlet_stats2(self.nx, self.ny, _ptr(self.types), self.tau, self.u_peak,
                                      self.rho_out, self.flags, _ptr(self.fs), _ptr(flow), cap,
                                      ctypes.byref(fin), ctypes.byref(dp), ctypes.byref(th),
                                      ctypes.byref(dg), ctypes.byref(m), ctypes.byref(p2))
        if n < 0:
            raise ValueError(f"oracle outlet_stats2 failed (rc={n})")
        return Stats2(flow[:n].copy(), fin.value, dp.value, th.value, dg.value, m.value, p2.value)

    def shape_update(self, frac=0.01, seed=0, band_x=2, band_y=1, criterion=CRIT_PAPER,
                     reinit=WARM, field=None) -> ShapeResult:
        """Exchange step on `field` = (rho, ux, uy) (default: this state's
        moments); updates types and reinitialises fs."""
        rho, ux, uy = field if field is not None else self.macro()
        rho = np.ascontiguousarray(rho, np.float64)
        ux = np.ascontiguousarray(ux, np.float64)
        uy = np.ascontiguousarray(uy, np.float64)
        cap = self.nx * self.ny
        rem = np.zeros(cap, np.int64)
        add = np.zeros(cap, np.int64)
        mr, ma = ctypes.c_double(), ctypes.c_double()
        nb, na = ctypes.c_int64(), ctypes.c_int64()
        k = _load().orc_shape_update(self.nx, self.ny, _ptr(self.types), _ptr(rho), _ptr(ux),
                                     _ptr(uy), float(frac), ctypes.c_uint64(seed & (2**64 - 1)),
                                     int(band_x), int(band_y), int(criterion), int(reinit),
                                     _ptr(self.fs), _ptr(rem), _ptr(add), cap,
                                     ctypes.byref(mr), ctypes.byref(ma), ctypes.byref(nb),
                                     ctypes.byref(na))
        if k < 0:
            raise ValueError(f"oracle shape_update failed (rc={k})")
        return ShapeResult(k, rem[:k].copy(), add[:k].copy(), mr.value, ma.value, nb.value,
                           na.value)


def shape_select(types, rho, ux, uy, frac=0.01, seed=0, band_x=2, band_y=1,
                 criterion=CRIT_PAPER):
    """Selection only (no state): returns (new_types, ShapeResult)."""
    t = np.ascontiguousarray(types, np.uint8).copy()
    lat = Lattice.__new__(Lattice)
    lat.types = t
    lat.ny, lat.nx = t.shape
    lat.fs = np.zeros((9, lat.ny, lat.nx))
    r = lat.shape_update(frac, seed, band_x, band_y, criterion, WARM, field=(rho, ux, uy))
    return lat.types, r
