#!/usr/bin/env python3
"""Benchmark of the LBM shape-optimisation hot path on one MI355X.

One benchmark step is one iteration of the optimisation loop (Sec. 2.3):
exchange step (Sec. 2.2) -> LBM solve to steady state (residual < tol, with a
step cap) -> outlet reductions (Eq. 4, Eqs. 9-11).  Before the warm-up the
lattice is brought from rest to steady state (untimed).

value  = lattice updates per second over the timed steps (all nx*ny cells,
         MLUPS), whole-job wall time between two device synchronisations.
roofline: the sweep kernel.  Algorithmic bytes per time step
         = 18 * s * N_nonsolid + N  (each non-solid population read and
         written once, s bytes each, plus one cell byte per cell); a launch
         advances steps_per_launch steps, so bytes per launch = that times
         the per-step figure.  Divided by the mean launch time of the sweeps
         inside the timed region, measured with HIP events recorded on the
         handle's stream around each residual-check interval's launches.
cpu_baseline: the FP64 oracle on the same lattice, a bounded number of steps.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "MLUPS + % HBM roofline (D2Q9 1024x512); p50/p99 solve latency, mixed load"
HBM_PEAK_GBS = 8000.0

# HBM bytes per time step of the plain sweep launches, from rocprofv3
# FETCH_SIZE / WRITE_SIZE (scaled by a plain copy of known size) of this
# build's kernels; profiles/sweep_tb_float_distributor-1024x512.txt.  Keyed by
# (workload, storage precision, kernel); reported as null for anything else
# and must be re-measured whenever the kernel changes.
MEASURED_TRAFFIC_PER_STEP = {
    ("distributor-1024x512-L3", "f32", "tb_kernel"): 14.902e6 / 8,
}


def workloads():
    from paper_1303_0107_amd import inputs as I
    return {w.name: w for w in (I.HEADLINE_1024x512, I.CHANNEL_1024x512, I.CORRECTNESS_128x64,
                                 I.PRECISION_2048x1024, I.CHANNEL_4096x2048)}


def copy_ceiling(nbytes: int = 1 << 28):
    """Device-to-device copy of nbytes with torch (a plain copy kernel of
    known size); returns the best read+write GB/s of 5 timed copies."""
    import torch
    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    b.copy_(a)
    best = 0.0
    for _ in range(5):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        b.copy_(a)
        e1.record()
        e1.synchronize()
        best = max(best, 2 * nbytes / (e0.elapsed_time(e1) * 1e-3) / 1e9)
    del a, b
    return best


def cpu_baseline(types, w, seconds: float):
    import oracle
    lat = oracle.Lattice(types, w.tau, w.u_peak)
    t0 = time.perf_counter()
    lat.run(50, 0.0, 50)
    dt = time.perf_counter() - t0
    steps = max(10, int(seconds / max(dt / 50, 1e-9)))
    lat = oracle.Lattice(types, w.tau, w.u_peak)
    t0 = time.perf_counter()
    lat.run(steps, 0.0, 100)
    dt = time.perf_counter() - t0
    return {"value": types.size * steps / dt / 1e6, "unit": "MLUPS",
            "cores": oracle.num_threads(), "kind": "oracle",
            "sample": f"{steps} FP64 time steps of the {w.name} lattice from rest "
                      f"({dt:.1f} s), residual checks every 100 steps"}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5, help="timed optimisation iterations")
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--precision", choices=["f32", "f64", "f16", "bf16"], default="f32",
                    help="population storage (f64: double storage and arithmetic; f32: float "
                         "storage, double arithmetic; f16/bf16: 16-bit storage, float arithmetic)")
    ap.add_argument("--workload", default="distributor-1024x512-L3")
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--cap", type=int, default=200000, help="step cap per solve")
    ap.add_argument("--settle-cap", type=int, default=None,
                    help="step cap of the untimed solve from rest (default: workload's)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu", action="store_true")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(the method's sharding is described in DESIGN.md)", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    from paper_1303_0107_amd import lbm

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 1
    torch.cuda.set_device(0)
    w = workloads()[args.workload]
    types = w.types()
    N = types.size
    nns = int(np.count_nonzero(types))
    prec = {"f64": lbm.LBM_F64, "f32": lbm.LBM_F32, "f16": lbm.LBM_F32_S_F16,
            "bf16": lbm.LBM_F32_S_BF16}[args.precision]
    s_bytes = {"f64": 8, "f32": 4, "f16": 2, "bf16": 2}[args.precision]
    arith = "f64" if args.precision in ("f64", "f32") else "f32"
    frac = w.extra.get("frac", 0.01)
    k = 100

    print(f"# workload {w.name} {w.nx}x{w.ny} non-solid {nns} precision {args.precision}",
          file=sys.stderr, flush=True)
    copy_gbs = copy_ceiling()
    lat = lbm.Lattice(types, w.tau, w.u_peak, precision=prec)
    t0 = time.perf_counter()
    settle_cap = args.settle_cap if args.settle_cap is not None else w.extra.get("cap0", 500000)
    rc, settle_steps, res = lat.run(settle_cap, args.tol, k)
    print(f"# settle: rc={rc} steps={settle_steps} r={res:.3e} "
          f"({time.perf_counter() - t0:.1f} s)", file=sys.stderr, flush=True)

    def one_step(seed):
        r, _, _ = lat.shape_update(frac=frac, seed=seed)
        rc, n, res = lat.run(args.cap, args.tol, k)
        flow, st = lat.stats()
        return n, res, flow, st, r

    for i in range(args.warmup):
        one_step(1000 + i)
    torch.cuda.synchronize()
    lat.profile_sweeps(True)
    sweeps = 0
    t0 = time.perf_counter()
    last = None
    for i in range(args.steps):
        n, res, flow, st, r = one_step(i + 1)
        sweeps += n
        last = (n, res, flow, st, r)
        print(f"# step {i}: k_eff={r.k_eff} sweeps={n} r={res:.2e} dp={st.dp:.6e} "
              f"theta={st.theta:.6f} dg={st.dg:.3e}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    timed_steps, launches, sweep_ms = lat.profile_sweeps(False)

    mlups = N * sweeps / wall / 1e6
    bytes_per_step = 18 * s_bytes * nns + N
    steps_per_launch = timed_steps / max(launches, 1)
    bytes_per_launch = bytes_per_step * steps_per_launch
    avg_ms = sweep_ms / max(launches, 1)
    achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9
    n, res, flow, st, r = last
    spread = float((flow.max() - flow.min()) / flow.mean()) if len(flow) else 0.0
    kernel = "tb_kernel" if steps_per_launch > 1.0 else "step_kernel"
    per_step = MEASURED_TRAFFIC_PER_STEP.get((w.name, args.precision, kernel))
    traffic = round(per_step * steps_per_launch) if per_step else None
    out = {
        "metric": METRIC,
        "value": round(mlups, 2),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall / args.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": arith,
        "data": "synthetic",
        "config": {
            "workload": w.name, "nx": w.nx, "ny": w.ny, "non_solid_cells": nns,
            "tau": w.tau, "u_peak": w.u_peak, "storage": args.precision, "arithmetic": arith,
            "step": f"exchange (frac {frac}) + solve to r<{args.tol:g} (cap {args.cap}, "
                    f"check every {k}) + outlet stats",
            "sweeps_timed": sweeps, "mflups": round(nns * sweeps / wall / 1e6, 2),
            "last_dp": st.dp, "last_theta": st.theta, "last_dg": st.dg,
            "last_spread": spread, "last_residual": res,
        },
        "roofline": {
            "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
            "kernel": kernel + f" ({args.precision} storage)",
            "bytes_per_step": bytes_per_step, "steps_per_launch": round(steps_per_launch, 3),
            "bytes_per_launch": round(bytes_per_launch), "launches": launches,
            "avg_launch_us": round(avg_ms * 1e3, 3),
            "copy_ceiling_GBs": round(copy_gbs, 1),
            "frac_of_copy_ceiling": round(achieved / copy_gbs, 4),
        },
    }
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(types, w, args.cpu_seconds)
    lat.close()
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
