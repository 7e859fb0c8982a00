"""ctypes binding of the C ABI in include/lbm.h (argument marshalling only).

Every function here forwards to the HIP library liblbm.so built in this
package directory; none computes anything itself.  If the library is missing
the first call raises: there is no fallback path.

PyTorch is only used to supply the HIP stream (torch.cuda.current_stream) and,
optionally, device memory; the library owns its own buffers.
"""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "liblbm.so")
HEADER_PATH = os.path.join(os.path.dirname(_PKG), "include", "lbm.h")

LBM_OK, LBM_NOT_CONVERGED = 0, 1
LBM_EINVAL, LBM_ENOMEM, LBM_EHIP, LBM_EUNSTABLE = -1, -2, -3, -4
LBM_SOLID, LBM_FLUID, LBM_INLET, LBM_OUTLET = 0, 1, 2, 3
LBM_F64, LBM_F32, LBM_F32_S_F16, LBM_F32_S_BF16 = 0, 1, 2, 3
LBM_WARM, LBM_COLD = 0, 1
LBM_CRIT_PAPER, LBM_CRIT_SPEED = 0, 1
LBM_REQ_SOLVE, LBM_REQ_OPTIMIZE = 0, 1
LBM_NEUMANN_OUTLET, LBM_SYMMETRY_TOP = 1, 2
LBM_TB_DENSE, LBM_TB_COMPACT, LBM_TB_INPLACE = 0, 1, 2


class LbmError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"lbm error {code}: {msg}")
        self.code = code


class lbm_geometry_desc(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("levels", ctypes.c_int32),
                ("widths", ctypes.c_int32 * 9), ("tau", ctypes.c_double),
                ("u_peak", ctypes.c_double), ("rho_out", ctypes.c_double),
                ("precision", ctypes.c_int32), ("flags", ctypes.c_int32)]


class lbm_stats(ctypes.Structure):
    _fields_ = [("n_outlets", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("n_fluid", ctypes.c_int64), ("n_nonsolid", ctypes.c_int64),
                ("flow_in", ctypes.c_double), ("dp", ctypes.c_double),
                ("theta", ctypes.c_double), ("dg", ctypes.c_double),
                ("flow_ave", ctypes.c_double), ("mass", ctypes.c_double),
                ("residual", ctypes.c_double), ("steps", ctypes.c_int64),
                ("flow_p2", ctypes.c_double)]


class lbm_shape_params(ctypes.Structure):
    _fields_ = [("frac", ctypes.c_double), ("seed", ctypes.c_uint64),
                ("band_x", ctypes.c_int32), ("band_y", ctypes.c_int32),
                ("criterion", ctypes.c_int32), ("reinit", ctypes.c_int32)]


class lbm_shape_result(ctypes.Structure):
    _fields_ = [("k_eff", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("n_cand_fluid", ctypes.c_int64), ("n_cand_solid", ctypes.c_int64),
                ("n_fluid_before", ctypes.c_int64), ("n_fluid_after", ctypes.c_int64),
                ("mass_removed", ctypes.c_double), ("mass_added", ctypes.c_double)]


class lbm_server_config(ctypes.Structure):
    _fields_ = [("hbm_budget", ctypes.c_size_t), ("max_sessions", ctypes.c_int32),
                ("quantum", ctypes.c_int32), ("variant", ctypes.c_int32),
                ("order", ctypes.c_int32)]


class lbm_request(ctypes.Structure):
    _fields_ = [("geom", lbm_geometry_desc), ("kind", ctypes.c_int32),
                ("iterations", ctypes.c_int32), ("solve_steps", ctypes.c_int64),
                ("steps_per_iteration", ctypes.c_int64), ("shape", lbm_shape_params)]


class lbm_result(ctypes.Structure):
    _fields_ = [("id", ctypes.c_uint64), ("status", ctypes.c_int32),
                ("iterations_done", ctypes.c_int32), ("steps", ctypes.c_int64),
                ("cells", ctypes.c_int64), ("digest", ctypes.c_uint64),
                ("t_submit", ctypes.c_double), ("t_admit", ctypes.c_double),
                ("t_done", ctypes.c_double), ("stats", lbm_stats)]


class lbm_server_stats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("completed", ctypes.c_int64),
                ("rejected", ctypes.c_int64), ("active", ctypes.c_int64),
                ("queued", ctypes.c_int64), ("rounds", ctypes.c_int64),
                ("cell_steps", ctypes.c_int64), ("nonsolid_cell_steps", ctypes.c_int64),
                ("busy_seconds", ctypes.c_double), ("admit_seconds", ctypes.c_double),
                ("sweep_seconds", ctypes.c_double), ("event_seconds", ctypes.c_double),
                ("peak_bytes", ctypes.c_size_t), ("exchange_seconds", ctypes.c_double),
                ("exchanges", ctypes.c_int64), ("exchange_calls", ctypes.c_int64)]


_lib = None


def declared_functions() -> list[str]:
    """Names of the functions include/lbm.h declares."""
    txt = open(HEADER_PATH).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(lbm_[a-z_]+)\s*\(", txt)))


def load() -> ctypes.CDLL:
    """Load liblbm.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"HIP library {LIB_PATH} is not built; run __graft_entry__.build()")
    lib = ctypes.CDLL(LIB_PATH)
    P, i32, i64, f64, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_size_t
    H = ctypes.c_void_p
    sig = {
        "lbm_create_geometry": (ctypes.c_int, [P, P, P, ctypes.POINTER(H)]),
        "lbm_run_to_steady": (ctypes.c_int, [H, i64, f64, i32, P, P]),
        "lbm_outlet_stats": (ctypes.c_int, [H, P, i32, P]),
        "lbm_shape_update": (ctypes.c_int, [H, P, P, P]),
        "lbm_last_exchange": (ctypes.c_int, [H, P, P, i32]),
        "lbm_get_mask": (ctypes.c_int, [H, P, sz]),
        "lbm_get_macro": (ctypes.c_int, [H, P, P, P, sz]),
        "lbm_get_state": (ctypes.c_int, [H, P, sz]),
        "lbm_set_state": (ctypes.c_int, [H, P, sz]),
        "lbm_footprint_bytes": (sz, [P]),
        "lbm_device_bytes": (ctypes.c_int, [H, P]),
        "lbm_destroy": (None, [H]),
        "lbm_last_error": (ctypes.c_char_p, []),
        "lbm_bench_sweep": (ctypes.c_int, [H, i32, P]),
        "lbm_profile_sweeps": (ctypes.c_int, [H, i32, P, P, P]),
        "lbm_tb_variant_count": (i32, [i32]),
        "lbm_tb_variant_info": (ctypes.c_int, [i32, i32, P, P, P, P]),
        "lbm_tb_variant_kind": (ctypes.c_int, [i32, i32, P, P]),
        "lbm_set_tb_variant": (ctypes.c_int, [H, i32]),
        "lbm_autotune": (ctypes.c_int, [H, i32, P, P, i32]),
        "lbm_batch_create": (ctypes.c_int, [P, i32, P, ctypes.POINTER(H)]),
        "lbm_batch_run": (ctypes.c_int, [H, i64, P]),
        "lbm_batch_configure": (ctypes.c_int, [H, i32, i32]),
        "lbm_batch_tune": (ctypes.c_int, [H, i32, P, P, P, i32]),
        "lbm_batch_info": (ctypes.c_int, [H, P, P, P]),
        "lbm_batch_destroy": (None, [H]),
        "lbm_batch_set_graphs": (ctypes.c_int, [H, i32]),
        "lbm_state_digest": (ctypes.c_int, [H, P]),
        "lbm_server_create": (ctypes.c_int, [P, P, ctypes.POINTER(H)]),
        "lbm_server_submit": (ctypes.c_int, [H, P, P]),
        "lbm_server_poll": (ctypes.c_int, [H, P, i32, i32]),
        "lbm_server_drain": (ctypes.c_int, [H]),
        "lbm_server_stats_get": (ctypes.c_int, [H, P]),
        "lbm_server_destroy": (None, [H]),
        "lbm_precision_info": (ctypes.c_int, [i32, P, P]),
        "lbm_outlet_stats_noalloc": (ctypes.c_int, [H, P, i32, P]),
        "lbm_get_tb_variant": (ctypes.c_int, [H, P]),
        "lbm_shape_update_many": (ctypes.c_int, [P, P, i32, P, P]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(rc: int) -> int:
    if rc < 0:
        raise LbmError(rc, load().lbm_last_error().decode())
    return rc


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def current_stream_handle():
    """hipStream_t of torch's current stream (None without a GPU)."""
    import torch
    if not torch.cuda.is_available():
        return None
    return torch.cuda.current_stream().cuda_stream


def make_desc(nx, ny, tau, u_peak, rho_out=1.0, precision=LBM_F64, levels=0, widths=None,
              flags=0):
    d = lbm_geometry_desc()
    d.nx, d.ny, d.levels = int(nx), int(ny), int(levels)
    for k, w in enumerate(widths or []):
        d.widths[k] = int(w)
    d.tau, d.u_peak, d.rho_out = float(tau), float(u_peak), float(rho_out)
    d.precision = int(precision)
    d.flags = int(flags)
    return d


def lbm_create_geometry(desc: lbm_geometry_desc, cell_types: np.ndarray | None = None,
                        hip_stream=None):
    lib = load()
    h = ctypes.c_void_p()
    types_ptr = None
    if cell_types is not None:
        cell_types = np.ascontiguousarray(cell_types, np.uint8)
        if cell_types.shape != (desc.ny, desc.nx):
            raise ValueError("cell_types must have shape (ny, nx)")
        types_ptr = _p(cell_types)
    _check(lib.lbm_create_geometry(ctypes.byref(desc), types_ptr, hip_stream, ctypes.byref(h)))
    return h


def lbm_run_to_steady(h, max_steps: int, tol: float = 0.0, check_every: int = 100):
    """Returns (status, steps_done, residual); status LBM_OK,
    LBM_NOT_CONVERGED or LBM_EUNSTABLE (the latter is returned, not raised)."""
    lib = load()
    steps = ctypes.c_int64(0)
    res = ctypes.c_double(0.0)
    rc = lib.lbm_run_to_steady(h, int(max_steps), float(tol), int(check_every),
                               ctypes.byref(steps), ctypes.byref(res))
    if rc < 0 and rc != LBM_EUNSTABLE:
        _check(rc)
    return rc, steps.value, res.value


def lbm_outlet_stats(h, flow_cap: int = 1024):
    lib = load()
    flow = np.zeros(max(flow_cap, 1), np.float64)
    s = lbm_stats()
    _check(lib.lbm_outlet_stats(h, _p(flow), int(flow_cap), ctypes.byref(s)))
    return flow[:s.n_outlets].copy(), s


def lbm_outlet_stats_noalloc(h, flow_cap: int = 1024):
    """lbm_outlet_stats without allocation (fixed per-GPU device scratch)."""
    lib = load()
    flow = np.zeros(max(flow_cap, 1), np.float64)
    s = lbm_stats()
    _check(lib.lbm_outlet_stats_noalloc(h, _p(flow), int(flow_cap), ctypes.byref(s)))
    return flow[:s.n_outlets].copy(), s


def make_shape_params(frac=0.01, seed=0, band_x=2, band_y=1, criterion=LBM_CRIT_PAPER,
                      reinit=LBM_WARM):
    p = lbm_shape_params()
    p.frac, p.seed = float(frac), int(seed) & (2 ** 64 - 1)
    p.band_x, p.band_y, p.criterion, p.reinit = int(band_x), int(band_y), int(criterion), int(reinit)
    return p


def lbm_shape_update(h, params: lbm_shape_params, rho_ux_uy=None):
    lib = load()
    r = lbm_shape_result()
    ptr = None
    if rho_ux_uy is not None:
        arr = np.ascontiguousarray(np.stack([np.asarray(a, np.float64) for a in rho_ux_uy]))
        ptr = _p(arr)
    _check(lib.lbm_shape_update(h, ctypes.byref(params), ptr, ctypes.byref(r)))
    return r


def lbm_shape_update_many(handles, params):
    """Exchange steps on many handles at once; returns (results, statuses)."""
    n = len(handles)
    hs = (ctypes.c_void_p * max(n, 1))(*handles)
    ps = (lbm_shape_params * max(n, 1))(*params)
    rs = (lbm_shape_result * max(n, 1))()
    st = (ctypes.c_int32 * max(n, 1))()
    rc = load().lbm_shape_update_many(hs, ps, n, rs, st)
    if rc < 0 and all(st[k] >= 0 for k in range(n)):
        _check(rc)
    return [rs[k] for k in range(n)], [st[k] for k in range(n)]


def lbm_last_exchange(h, cap: int):
    lib = load()
    rem = np.zeros(max(cap, 1), np.int64)
    add = np.zeros(max(cap, 1), np.int64)
    k = _check(lib.lbm_last_exchange(h, _p(rem), _p(add), int(cap)))
    return rem[:k].copy(), add[:k].copy()


def lbm_get_mask(h, nx: int, ny: int) -> np.ndarray:
    out = np.zeros((ny, nx), np.uint8)
    _check(load().lbm_get_mask(h, _p(out), out.size))
    return out


def lbm_get_macro(h, nx: int, ny: int):
    rho = np.zeros((ny, nx))
    ux = np.zeros((ny, nx))
    uy = np.zeros((ny, nx))
    _check(load().lbm_get_macro(h, _p(rho), _p(ux), _p(uy), rho.size))
    return rho, ux, uy


def lbm_get_state(h, nx: int, ny: int) -> np.ndarray:
    f = np.zeros((9, ny, nx))
    _check(load().lbm_get_state(h, _p(f), f.size))
    return f


def lbm_set_state(h, f: np.ndarray) -> None:
    f = np.ascontiguousarray(f, np.float64)
    _check(load().lbm_set_state(h, _p(f), f.size))


def lbm_footprint_bytes(desc: lbm_geometry_desc) -> int:
    return int(load().lbm_footprint_bytes(ctypes.byref(desc)))


def lbm_device_bytes(h) -> int:
    n = ctypes.c_size_t(0)
    _check(load().lbm_device_bytes(h, ctypes.byref(n)))
    return int(n.value)


def lbm_destroy(h) -> None:
    if h:
        load().lbm_destroy(h)


def lbm_last_error() -> str:
    return load().lbm_last_error().decode()


def lbm_bench_sweep(h, steps: int) -> float:
    ms = ctypes.c_double(0.0)
    _check(load().lbm_bench_sweep(h, int(steps), ctypes.byref(ms)))
    return ms.value


def lbm_profile_sweeps(h, enable: bool):
    """Returns (steps, kernel launches, total_ms) recorded so far."""
    n = ctypes.c_int64(0)
    k = ctypes.c_int64(0)
    ms = ctypes.c_double(0.0)
    _check(load().lbm_profile_sweeps(h, int(bool(enable)), ctypes.byref(n), ctypes.byref(k),
                                     ctypes.byref(ms)))
    return n.value, k.value, ms.value


def lbm_precision_info(precision: int) -> tuple[int, int]:
    """(bytes per stored population value, bytes of the update's arithmetic)."""
    sb, ab = ctypes.c_int32(), ctypes.c_int32()
    _check(load().lbm_precision_info(int(precision), ctypes.byref(sb), ctypes.byref(ab)))
    return sb.value, ab.value


def lbm_tb_variant_count(precision: int) -> int:
    return int(load().lbm_tb_variant_count(int(precision)))


def lbm_tb_variant_info(precision: int, variant: int):
    """(rows, halo, tile_w, tile_h) of a compiled region shape."""
    v = [ctypes.c_int32(0) for _ in range(4)]
    _check(load().lbm_tb_variant_info(int(precision), int(variant),
                                      *[ctypes.byref(x) for x in v]))
    return tuple(x.value for x in v)


def lbm_tb_variant_kind(precision: int, variant: int):
    """(kind, LDS bytes per workgroup) of a compiled region shape; kind is
    LBM_TB_DENSE, LBM_TB_COMPACT or LBM_TB_INPLACE."""
    v = [ctypes.c_int32(0) for _ in range(2)]
    _check(load().lbm_tb_variant_kind(int(precision), int(variant),
                                      *[ctypes.byref(x) for x in v]))
    return tuple(x.value for x in v)


def lbm_get_tb_variant(h) -> int:
    """The region shape in use (-1: one launch per step)."""
    v = ctypes.c_int32()
    _check(load().lbm_get_tb_variant(h, ctypes.byref(v)))
    return v.value


def lbm_set_tb_variant(h, variant: int) -> None:
    _check(load().lbm_set_tb_variant(h, int(variant)))


def lbm_autotune(h, trial_steps: int, n_variants: int):
    """Returns (best shape, ms per step of each shape)."""
    best = ctypes.c_int32(0)
    ms = np.zeros(n_variants, dtype=np.float64)
    _check(load().lbm_autotune(h, int(trial_steps), ctypes.byref(best), _p(ms), n_variants))
    return best.value, ms


def lbm_batch_create(handles, stream=None):
    arr = (ctypes.c_void_p * len(handles))(*handles)
    out = ctypes.c_void_p()
    _check(load().lbm_batch_create(ctypes.cast(arr, ctypes.c_void_p), len(handles), stream,
                                   ctypes.byref(out)))
    return out


def lbm_batch_run(b, steps: int) -> float:
    """Advance every member; returns the elapsed milliseconds of the launches."""
    ms = ctypes.c_double(0.0)
    _check(load().lbm_batch_run(b, int(steps), ctypes.byref(ms)))
    return ms.value


def lbm_batch_configure(b, variant: int, order: int) -> None:
    _check(load().lbm_batch_configure(b, int(variant), int(order)))


def lbm_batch_tune(b, trial_steps: int, n_variants: int):
    """n_variants = shape count + 1 (the single-step mode).  Returns (best
    variant, best order, ms per step of configuration 2*variant+order)."""
    bv = ctypes.c_int32(0)
    bo = ctypes.c_int32(0)
    ms = np.zeros(2 * n_variants, dtype=np.float64)
    _check(load().lbm_batch_tune(b, int(trial_steps), ctypes.byref(bv), ctypes.byref(bo),
                                 _p(ms), 2 * n_variants))
    return bv.value, bo.value, ms


def lbm_batch_info(b):
    """(tiles per launch, steps per launch, summed non-solid cells)."""
    items = ctypes.c_int64(0)
    spl = ctypes.c_int32(0)
    cells = ctypes.c_int64(0)
    _check(load().lbm_batch_info(b, ctypes.byref(items), ctypes.byref(spl), ctypes.byref(cells)))
    return items.value, spl.value, cells.value


def lbm_batch_destroy(b) -> None:
    load().lbm_batch_destroy(b)


def lbm_batch_set_graphs(b, enable: bool) -> None:
    _check(load().lbm_batch_set_graphs(b, int(bool(enable))))


def lbm_state_digest(h) -> int:
    d = ctypes.c_uint64(0)
    _check(load().lbm_state_digest(h, ctypes.byref(d)))
    return d.value


def make_request(nx, ny, levels, widths, tau, u_peak, precision=LBM_F32, kind=LBM_REQ_SOLVE,
                 solve_steps=500, iterations=0, steps_per_iteration=0, frac=0.01, seed=0,
                 band_x=2, band_y=1, criterion=LBM_CRIT_PAPER, reinit=LBM_WARM, rho_out=1.0):
    r = lbm_request()
    r.geom = make_desc(nx, ny, tau, u_peak, rho_out, precision, levels, widths)
    r.kind = int(kind)
    r.iterations = int(iterations)
    r.solve_steps = int(solve_steps)
    r.steps_per_iteration = int(steps_per_iteration)
    r.shape = make_shape_params(frac, seed, band_x, band_y, criterion, reinit)
    return r


class Server:
    """Owning wrapper of a request server (worker thread in the library)."""

    def __init__(self, hbm_budget: int, max_sessions: int = 64, quantum: int = 40,
                 variant: int = -1, order: int = 1, stream=None):
        cfg = lbm_server_config(int(hbm_budget), int(max_sessions), int(quantum), int(variant),
                                int(order))
        if stream is None:
            stream = current_stream_handle()
        out = ctypes.c_void_p()
        _check(load().lbm_server_create(ctypes.byref(cfg), stream, ctypes.byref(out)))
        self.s = out

    def submit(self, req: lbm_request) -> int:
        i = ctypes.c_uint64(0)
        _check(load().lbm_server_submit(self.s, ctypes.byref(req), ctypes.byref(i)))
        return i.value

    def poll(self, cap: int = 256, wait_ms: int = 0):
        arr = (lbm_result * max(cap, 1))()
        n = _check(load().lbm_server_poll(self.s, arr, int(cap), int(wait_ms)))
        return [arr[k] for k in range(n)]

    def drain(self) -> None:
        _check(load().lbm_server_drain(self.s))

    def stats(self) -> lbm_server_stats:
        st = lbm_server_stats()
        _check(load().lbm_server_stats_get(self.s, ctypes.byref(st)))
        return st

    def close(self):
        if self.s:
            load().lbm_server_destroy(self.s)
            self.s = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Lattice:
    """Owning wrapper of one handle."""

    def __init__(self, types: np.ndarray | None, tau: float, u_peak: float, rho_out: float = 1.0,
                 precision: int = LBM_F64, nx: int | None = None, ny: int | None = None,
                 levels: int = 0, widths=None, stream=None, flags: int = 0):
        if types is not None:
            ny, nx = types.shape
        self.nx, self.ny = int(nx), int(ny)
        self.precision = int(precision)
        self.desc = make_desc(self.nx, self.ny, tau, u_peak, rho_out, precision, levels, widths,
                              flags)
        if stream is None:
            stream = current_stream_handle()
        self.h = lbm_create_geometry(self.desc, types, stream)

    def close(self):
        if self.h:
            lbm_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def run(self, max_steps, tol=0.0, check_every=100):
        return lbm_run_to_steady(self.h, max_steps, tol, check_every)

    def device_bytes(self):
        return lbm_device_bytes(self.h)

    def stats(self, flow_cap=1024):
        return lbm_outlet_stats(self.h, flow_cap)

    def shape_update(self, frac=0.01, seed=0, band_x=2, band_y=1, criterion=LBM_CRIT_PAPER,
                     reinit=LBM_WARM, field=None):
        p = make_shape_params(frac, seed, band_x, band_y, criterion, reinit)
        r = lbm_shape_update(self.h, p, field)
        rem, add = lbm_last_exchange(self.h, max(r.k_eff, 1))
        return r, rem, add

    def mask(self):
        return lbm_get_mask(self.h, self.nx, self.ny)

    def macro(self):
        return lbm_get_macro(self.h, self.nx, self.ny)

    def state(self):
        return lbm_get_state(self.h, self.nx, self.ny)

    def set_state(self, f):
        lbm_set_state(self.h, f)

    def bench_sweep(self, steps):
        return lbm_bench_sweep(self.h, steps)

    def profile_sweeps(self, enable):
        return lbm_profile_sweeps(self.h, enable)

    def set_tb_variant(self, variant):
        lbm_set_tb_variant(self.h, variant)

    def autotune(self, trial_steps):
        return lbm_autotune(self.h, trial_steps, lbm_tb_variant_count(self.precision))

    def digest(self):
        return lbm_state_digest(self.h)


class Batch:
    """Owning wrapper of a batch; keeps its member Lattice objects alive."""

    def __init__(self, lattices, stream=None):
        self.members = list(lattices)
        if stream is None:
            stream = current_stream_handle()
        self.precision = self.members[0].precision if self.members else LBM_F64
        self.b = lbm_batch_create([m.h for m in self.members], stream)

    def close(self):
        if self.b:
            lbm_batch_destroy(self.b)
            self.b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def run(self, steps):
        return lbm_batch_run(self.b, steps)

    def configure(self, variant, order):
        lbm_batch_configure(self.b, variant, order)

    def tune(self, trial_steps):
        return lbm_batch_tune(self.b, trial_steps, lbm_tb_variant_count(self.precision) + 1)

    def info(self):
        return lbm_batch_info(self.b)
