#!/usr/bin/env python3
"""Benchmark of the LBM shape-optimisation hot path on one MI355X.

One benchmark step is one iteration of the optimisation loop (Sec. 2.3):
exchange step (Sec. 2.2) -> LBM solve to steady state (residual < tol, with a
step cap) -> outlet reductions (Eq. 4, Eqs. 9-11).  Before the warm-up the
lattice is brought from rest to steady state (untimed).

value  = lattice updates per second over the timed steps (all nx*ny cells,
         MLUPS), whole-job wall time between two device synchronisations;
         mflups counts the non-solid cells only.
roofline: the sweep kernel.  Algorithmic bytes per time step
         = 18 * s * N_nonsolid + N  (each non-solid population read and
         written once, s bytes each, plus one cell byte per cell); a launch
         advances steps_per_launch steps, so bytes per launch = that times
         the per-step figure.  Divided by the mean launch time of the sweeps
         inside the timed region, measured with HIP events recorded on the
         handle's stream around each residual-check interval's launches.
         With temporal blocking a launch moves far fewer bytes than that
         (the populations cross HBM once per launch, not once per step), so
         this is an effective bandwidth; the measured HBM bytes per launch
         (rocprofv3 counters) over the same launch time are reported beside
         it, and so is the kernel's actual limiter, the vector ALU issue rate
         (measured VALU instructions per launch over the launch time, against
         the chip's non-packed rate).
Default legs (--legs): the headline optimisation loop; the all-fluid
1024x512 channel (sweeps only: the workload the HBM-roofline target is set
on); a short serving run (Poisson arrivals, p50/p99 latency).
cpu_baseline: the FP64 oracle on the same lattice, a bounded number of steps,
on every host thread and on one.
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

# HBM bytes of one full launch (halo = steps per launch) of the blocked
# sweep, from rocprofv3 FETCH_SIZE / WRITE_SIZE (scaled by a plain copy of
# known size) of this build's kernels; profiles/sweep_tb_*.txt.  Keyed by
# (workload, storage precision, region shape); reported as null for anything
# else and must be re-measured whenever the kernel changes.  A launch moves
# about the same bytes whatever its step count (it loads its region and
# stores its tile once), and the last launch of each check interval also
# reads and writes u_prev (two FP64 planes, 32 B per non-solid cell), so the
# reported traffic per launch is full + 32 B * N_ns / (launches per interval).
MEASURED_TRAFFIC_PER_FULL_LAUNCH = {
    # profiles/sweep_tb_float_distributor-1024x512.txt: shape 5 (32x64 dense
    # regions, 9 steps per launch, 236 active tiles), shape 1 (32x64 dense, 8
    # steps per launch, 234 tiles), shape 0 (32x64 compacted)
    ("distributor-1024x512-L3", "f32", 5): 8.486e6,
    ("distributor-1024x512-L3", "f32", 1): 8.403e6,
    ("distributor-1024x512-L3", "f32", 0): 8.474e6,
    # profiles/sweep_tb_double_distributor-1024x512.txt: shape 3 (32x64 in
    # place, 8 steps per launch), shape 0 (16x64 compacted, 4 steps per
    # launch), shape 1 (16x64 dense)
    ("distributor-1024x512-L3", "f64", 3): 18.718e6,
    ("distributor-1024x512-L3", "f64", 0): 13.163e6,
    ("distributor-1024x512-L3", "f64", 1): 13.133e6,
    # profiles/sweep_tb_float_channel-1024x512.txt: shape 4 (16x64 dense, 4
    # steps per launch), shape 3 (16x64 compacted), shapes 1 and 0 (32x64
    # dense and compacted, 8 steps per launch), shape 5 (32x64 dense, 9 steps)
    ("channel-1024x512", "f32", 4): 41.012e6,
    ("channel-1024x512", "f32", 3): 41.030e6,
    ("channel-1024x512", "f32", 1): 43.170e6,
    ("channel-1024x512", "f32", 0): 43.250e6,
    ("channel-1024x512", "f32", 5): 44.016e6,
    # profiles/sweep_tb_float_channel-4096x2048.txt, the same shapes
    ("channel-4096x2048", "f32", 4): 637.188e6,
    ("channel-4096x2048", "f32", 3): 640.631e6,
    ("channel-4096x2048", "f32", 1): 935.983e6,
    ("channel-4096x2048", "f32", 0): 936.164e6,
    ("channel-4096x2048", "f32", 5): 1027.100e6,
}
# The same for the batched kernel, per launch, keyed by (workload, storage,
# shape, order).
MEASURED_TRAFFIC_PER_LAUNCH = {
    # profiles/sweep_batch_float_batch-256-candidates.txt; shapes 0..5 temporal
    # blocking (0: 32x64 compacted, 1: 32x64 dense, 2: 32x64 compacted with
    # 4 steps per launch, 3: 16x64 compacted, 4: 16x64 dense, 5: 32x64 dense
    # with 9 steps per launch), 6 = one step per launch
    ("batch-256-candidates", "f32", 4, 1): 700.888e6,
    ("batch-256-candidates", "f32", 4, 0): 1366.060e6,
    ("batch-256-candidates", "f32", 3, 1): 700.887e6,
    ("batch-256-candidates", "f32", 3, 0): 1366.061e6,
    ("batch-256-candidates", "f32", 2, 1): 708.363e6,
    ("batch-256-candidates", "f32", 2, 0): 1090.876e6,
    ("batch-256-candidates", "f32", 1, 1): 709.157e6,
    ("batch-256-candidates", "f32", 1, 0): 1556.352e6,
    ("batch-256-candidates", "f32", 0, 1): 709.222e6,
    ("batch-256-candidates", "f32", 0, 0): 1556.446e6,
    ("batch-256-candidates", "f32", 5, 1): 708.557e6,
    ("batch-256-candidates", "f32", 5, 0): 1637.074e6,
    ("batch-256-candidates", "f32", 6, 1): 684.537e6,
    ("batch-256-candidates", "f32", 6, 0): 775.521e6,
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


def cpu_model() -> str:
    """The host CPU's model name (from /proc/cpuinfo)."""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_rate(types, w, seconds: float, threads: int | None):
    import oracle
    if threads:
        oracle.set_num_threads(threads)
    lat = oracle.Lattice(types, w.tau, w.u_peak)
    steps = 0
    t0 = time.perf_counter()
    while True:
        lat.run(100, 0.0, 100)
        steps += 100
        dt = time.perf_counter() - t0
        if dt >= seconds:
            break
    return types.size * steps / dt / 1e6, steps, dt, oracle.num_threads()


def cpu_baseline(types, w, seconds: float):
    """The oracle from rest on the same lattice, in chunks of 100 steps
    (residual check each) until `seconds` of wall time have passed: once on
    every host thread, once on a single thread."""
    import oracle
    # the host threads this process may use (the job's share of the host)
    all_threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count() or 1
    mlups, steps, dt, cores = _oracle_rate(types, w, seconds, all_threads)
    one, steps1, dt1, _ = _oracle_rate(types, w, seconds / 2, 1)
    oracle.set_num_threads(all_threads)
    nns = int((types != 0).sum())
    return {"value": mlups, "unit": "MLUPS", "cores": cores, "kind": "oracle",
            "sample": f"{steps} FP64 time steps of the {w.name} lattice from rest "
                      f"({dt:.1f} s), residual checks every 100 steps",
            "mflups": mlups * nns / types.size,
            "single_thread": {"value": one, "unit": "MLUPS", "cores": 1,
                              "sample": f"{steps1} time steps ({dt1:.1f} s)"},
            "single_thread_mflups": one * nns / types.size,
            "cpu_model": cpu_model(), "host_threads": all_threads,
            "nproc": os.cpu_count()}


BATCH_WORKLOAD = "batch-256-candidates"


def bench_batch(args) -> int:
    """Batched candidates: 256 uneven distributors advanced together.  One
    benchmark step = every candidate advanced by --batch-steps time steps
    (one batch run).  value = all cells of all candidates times steps over
    the wall time of the timed runs.  roofline: the batch kernel, algorithmic
    bytes per launch = steps per launch * sum over candidates of
    (18 s N_nonsolid + N), over the mean launch time (HIP events around each
    run's launches on the batch's stream, divided by its launch count)."""
    import numpy as np
    import torch

    from paper_1303_0107_amd import inputs as I
    from paper_1303_0107_amd import lbm

    prec = {"f64": lbm.LBM_F64, "f32": lbm.LBM_F32, "f16": lbm.LBM_F32_S_F16,
            "bf16": lbm.LBM_F32_S_BF16}[args.precision]
    s_bytes = {"f64": 8, "f32": 4, "f16": 2, "bf16": 2}[args.precision]
    arith = "f64" if args.precision == "f64" else "f32"
    cands = I.batch_candidates(count=args.batch_count, seed=4)
    types = [c.types() for c in cands]
    N = sum(t.size for t in types)
    nns = sum(int(np.count_nonzero(t)) for t in types)
    print(f"# {BATCH_WORKLOAD}: {len(cands)} lattices, {N} cells, {nns} non-solid, "
          f"precision {args.precision}", file=sys.stderr, flush=True)
    copy_gbs = copy_ceiling()
    lats = [lbm.Lattice(t, c.tau, c.u_peak, precision=prec) for t, c in zip(types, cands)]
    bt = lbm.Batch(lats)
    t0 = time.perf_counter()
    bv, bo, trial = bt.tune(args.tune_steps)
    print(f"# tuned in {time.perf_counter() - t0:.1f} s: shape {bv} order {bo}; ms/step "
          + " ".join(f"{x:.3f}" for x in trial), file=sys.stderr, flush=True)
    if bv < lbm.lbm_tb_variant_count(prec):
        rows, halo, tw, th = lbm.lbm_tb_variant_info(prec, bv)
        shape = {"kind": "temporal blocking", "rows": rows, "halo": halo, "tile": [tw, th],
                 "order": bo}
        kname = "tb_batch_kernel"
    else:
        shape = {"kind": "one step per launch", "block": [64, 4], "order": bo}
        kname = "step_batch_kernel"
    for _ in range(args.warmup):
        bt.run(args.batch_steps)
    torch.cuda.synchronize()
    launch_ms = 0.0
    t0 = time.perf_counter()
    for i in range(args.steps):
        ms = bt.run(args.batch_steps)
        launch_ms += ms
        print(f"# step {i}: {args.batch_steps} steps in {ms:.1f} ms", file=sys.stderr,
              flush=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    items, spl, _ = bt.info()
    launches_per_run = -(-args.batch_steps // spl)
    launches = launches_per_run * args.steps
    total_steps = args.batch_steps * args.steps
    mlups = N * total_steps / wall / 1e6
    bytes_per_step = 18 * s_bytes * nns + N
    avg_ms = launch_ms / launches
    bytes_per_launch = bytes_per_step * args.batch_steps / launches_per_run
    achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9
    flows = []
    for lat in lats[:4]:
        flow, st = lat.stats()
        flows.append(round(float(st.dp), 9))
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
            "workload": BATCH_WORKLOAD, "lattices": len(cands), "cells": N,
            "non_solid_cells": nns, "storage": args.precision, "arithmetic": arith,
            "step": f"every lattice advanced {args.batch_steps} time steps in one batch",
            "sizes": "nx 128..1024, ny 64..512 (multiples of 64), 2-4 levels, "
                     "tau U[0.55,1], u_peak U[0.02,0.06]",
            "mflups": round(nns * total_steps / wall / 1e6, 2),
            "tuned_shape": shape,
            "tune_ms_per_step": [round(x, 4) for x in trial],
            "dp_first_members": flows,
        },
        "roofline": {
            "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": MEASURED_TRAFFIC_PER_LAUNCH.get((BATCH_WORKLOAD, args.precision, bv, bo)),
            "kernel": f"{kname} ({args.precision} storage)",
            "bytes_per_step": bytes_per_step, "steps_per_launch": spl,
            "bytes_per_launch": round(bytes_per_launch), "launches": launches,
            "work_items_per_launch": items,
            "avg_launch_us": round(avg_ms * 1e3, 3),
            "copy_ceiling_GBs": round(copy_gbs, 1),
            "frac_of_copy_ceiling": round(achieved / copy_gbs, 4),
        },
    }
    hbm_and_limiter(out["roofline"], out["roofline"]["traffic"],
                    MEASURED_VALU_PER_LAUNCH.get((BATCH_WORKLOAD, args.precision, bv, bo)),
                    avg_ms)
    if not args.no_cpu:
        big = max(range(len(cands)), key=lambda i: types[i].size)
        out["cpu_baseline"] = cpu_baseline(types[big], cands[big], args.cpu_seconds)
    bt.close()
    for lat in lats:
        lat.close()
    print(json.dumps(out), flush=True)
    return 0


SERVE_WORKLOAD = "serve-poisson-50rps"


def serve_leg(args, rate: float, seconds: float):
    """Serving: Poisson arrivals of solve / optimise requests (FP32 and FP16
    offset storage) submitted in real time to the request server (continuous
    batching, admission by HBM footprint).  value = aggregate lattice updates
    per second (all cells of every request times its steps) over the wall
    time from the first arrival to the last completion; latency = completion
    minus submission per request, p50 / p99.  roofline: whole rounds (batched
    sweeps plus the host work of events), algorithmic bytes of the steps
    taken over the time spent in rounds -- a lower bound on the kernels'
    rate, not a kernel measurement.  Returns (result dict, failures)."""
    import numpy as np
    import torch

    from paper_1303_0107_amd import inputs as I
    from paper_1303_0107_amd import lbm

    reqs = I.serving_requests(rate=rate, seconds=seconds, seed=5)
    prec = {"f32": lbm.LBM_F32, "f16": lbm.LBM_F32_S_F16}
    s_bytes = {"f32": 4, "f16": 2}
    print(f"# serving: {len(reqs)} requests over {seconds} s at {rate}/s",
          file=sys.stderr, flush=True)
    crs = []
    nns = []
    for q in reqs:
        w = q.workload
        kind = lbm.LBM_REQ_SOLVE if q.kind == "solve" else lbm.LBM_REQ_OPTIMIZE
        crs.append(lbm.make_request(w.nx, w.ny, w.levels, w.widths, w.tau, w.u_peak,
                                    prec[q.storage], kind, solve_steps=q.solve_steps,
                                    iterations=q.iterations,
                                    steps_per_iteration=q.steps_per_iteration,
                                    frac=0.01, seed=q.seed))
    budget = int(args.hbm_budget_gb * (1 << 30))
    srv = lbm.Server(hbm_budget=budget, max_sessions=args.max_sessions, quantum=args.quantum,
                     variant=-1, order=1)
    # Warm-up, untimed: 24 requests of both storage forms at once (the
    # library's first calls load its code, and the server autotunes its batch
    # configuration on the first batch of 8 members of each form), then the
    # counters are taken as the baseline of the timed run.
    warm = I.serving_requests(rate=1000.0, seconds=0.05, seed=105)
    for q in warm[:24]:
        w = q.workload
        srv.submit(lbm.make_request(w.nx, w.ny, w.levels, w.widths, w.tau, w.u_peak,
                                    prec[q.storage], lbm.LBM_REQ_SOLVE, solve_steps=40))
    srv.drain()
    srv.poll(cap=64)
    st0 = srv.stats()
    torch.cuda.synchronize()
    results = {}
    ids = {}
    t0 = time.perf_counter()
    last_print = t0
    for k, q in enumerate(reqs):
        while True:
            now = time.perf_counter() - t0
            if now >= q.t:
                break
            for r in srv.poll(cap=256, wait_ms=max(1, int((q.t - now) * 1e3))):
                results[r.id] = r
        ids[srv.submit(crs[k])] = k
        if time.perf_counter() - last_print > 10:
            last_print = time.perf_counter()
            print(f"# t={last_print - t0:.0f}s submitted {k + 1} done {len(results)}",
                  file=sys.stderr, flush=True)
    srv.drain()
    for r in srv.poll(cap=len(reqs) + 8):
        results[r.id] = r
    wall = time.perf_counter() - t0
    st1 = srv.stats()
    srv.close()
    st = lbm.lbm_server_stats()  # the timed run's share of the counters
    for name, _ in lbm.lbm_server_stats._fields_:
        setattr(st, name, getattr(st1, name) - getattr(st0, name))
    st.peak_bytes = st1.peak_bytes
    res = [results[i] for i in sorted(results)]
    bad = [r for r in res if r.status != lbm.LBM_OK]
    lat = np.array([r.t_done - r.t_submit for r in res]) * 1e3
    queue = np.array([r.t_admit - r.t_submit for r in res]) * 1e3
    mlups = st.cell_steps / wall / 1e6
    # algorithmic bytes of the steps taken (per request: 18 s N_ns + N per step)
    algo = 0.0
    for r in res:
        q = reqs[ids[r.id]]
        algo += r.steps * (18 * s_bytes[q.storage] * r.stats.n_nonsolid + r.cells)
    achieved = algo / st.busy_seconds / 1e9 if st.busy_seconds > 0 else 0.0
    out = {
        "metric": METRIC,
        "value": round(mlups, 2),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": len(reqs),
        "warmup": 0,
        "ms_per_step": round(wall / max(len(reqs), 1) * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": SERVE_WORKLOAD, "requests": len(reqs),
            "arrivals": f"Poisson {rate}/s for {seconds} s, seed 5",
            "lattices": "nx = 64 round(256 2^U(0,4) / 64), ny = nx/2; generator as the "
                        "batched candidates",
            "mix": "FP32 / FP16 offset storage 50/50 (float arithmetic); solve 500 steps / "
                   "optimise 100 steps + 20 x (exchange step + 40 steps), 50/50",
            "hbm_budget_gb": args.hbm_budget_gb, "max_sessions": args.max_sessions,
            "quantum": args.quantum,
            "latency_ms": {"p50": round(float(np.percentile(lat, 50)), 2),
                           "p99": round(float(np.percentile(lat, 99)), 2),
                           "mean": round(float(lat.mean()), 2),
                           "max": round(float(lat.max()), 2)},
            "queue_ms": {"p50": round(float(np.percentile(queue, 50)), 2),
                         "p99": round(float(np.percentile(queue, 99)), 2)},
            "failed": len(bad), "rounds": st.rounds, "busy_seconds": round(st.busy_seconds, 3),
            "admit_seconds": round(st.admit_seconds, 3),
            "sweep_seconds": round(st.sweep_seconds, 3),
            "event_seconds": round(st.event_seconds, 3),
            "exchange_seconds": round(st.exchange_seconds, 3), "exchanges": st.exchanges,
            "exchange_calls": st.exchange_calls,
            "wall_seconds": round(wall, 3), "peak_bytes": st.peak_bytes,
            "mflups": round(st.nonsolid_cell_steps / wall / 1e6, 2),
        },
        "roofline": {
            "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
            "kernel": "server rounds (batched sweeps + event host work), not a single kernel",
        },
    }
    return out, len(bad)


def bench_serve(args) -> int:
    """The serving workload on its own (value = its aggregate MLUPS)."""
    from paper_1303_0107_amd import inputs as I
    out, bad = serve_leg(args, args.serve_rate, args.serve_seconds)
    out["latency_ms"] = out["config"]["latency_ms"]
    if not args.no_cpu:
        w = I.HEADLINE_1024x512
        out["cpu_baseline"] = cpu_baseline(w.types(), w, args.cpu_seconds)
    print(json.dumps(out), flush=True)
    return 0 if not bad else 1


# Vector ALU instructions (wave instructions, rocprofv3 SQ_INSTS_VALU) of one
# full launch of the blocked sweep, keyed like the traffic table, from the
# same profiles.  Each wave instruction occupies a SIMD for 4 cycles (64
# lanes on 16-wide SIMDs; packed FP32 is not used), so the chip issues at
# most 256 CUs x 4 SIMDs x 2.4 GHz / 4 = 614.4 G wave instructions per second.
MEASURED_VALU_PER_FULL_LAUNCH = {
    ("distributor-1024x512-L3", "f32", 5): 3.937e6,
    ("distributor-1024x512-L3", "f32", 1): 3.455e6,
    ("distributor-1024x512-L3", "f32", 0): 3.218e6,
    ("distributor-1024x512-L3", "f64", 3): 5.611e6,
    ("distributor-1024x512-L3", "f64", 1): 2.433e6,
    ("distributor-1024x512-L3", "f64", 0): 2.240e6,
    ("channel-1024x512", "f32", 4): 8.107e6,
    ("channel-1024x512", "f32", 3): 9.306e6,
    ("channel-1024x512", "f32", 1): 15.07e6,
    ("channel-1024x512", "f32", 0): 16.11e6,
    ("channel-1024x512", "f32", 5): 19.17e6,
    ("channel-4096x2048", "f32", 4): 125.8e6,
    ("channel-4096x2048", "f32", 3): 146.8e6,
    ("channel-4096x2048", "f32", 1): 235.3e6,
    ("channel-4096x2048", "f32", 0): 256.4e6,
    ("channel-4096x2048", "f32", 5): 296.9e6,
}
# The same for the batched kernel, per launch, keyed by (workload, storage,
# shape, order) like MEASURED_TRAFFIC_PER_LAUNCH.
MEASURED_VALU_PER_LAUNCH = {
    ("batch-256-candidates", "f32", 4, 1): 206.5e6,
    ("batch-256-candidates", "f32", 4, 0): 206.5e6,
    ("batch-256-candidates", "f32", 3, 1): 199.2e6,
    ("batch-256-candidates", "f32", 3, 0): 199.2e6,
    ("batch-256-candidates", "f32", 2, 1): 158.7e6,
    ("batch-256-candidates", "f32", 1, 1): 385.6e6,
    ("batch-256-candidates", "f32", 1, 0): 385.6e6,
    ("batch-256-candidates", "f32", 0, 1): 330.9e6,
    ("batch-256-candidates", "f32", 0, 0): 330.9e6,
    ("batch-256-candidates", "f32", 6, 1): 43.54e6,
    ("batch-256-candidates", "f32", 6, 0): 43.54e6,
}
VALU_PEAK_WAVE_INSTR_PER_S = 256 * 4 * 2.4e9 / 4


def hbm_and_limiter(roof: dict, traffic, valu, avg_ms: float) -> None:
    """Add the measured HBM rate and the ALU-issue bound to a roofline dict."""
    roof["effective"] = "algorithmic bytes of every step a launch advances over the launch " \
                        "time (with temporal blocking, above what HBM carries)"
    if traffic:
        gbs = traffic / (avg_ms * 1e-3) / 1e9
        roof["hbm_measured_GBs"] = round(gbs, 1)
        roof["hbm_measured_frac"] = round(gbs / HBM_PEAK_GBS, 4)
    else:
        roof["hbm_measured_GBs"] = None
        roof["hbm_measured_frac"] = None
    if valu:
        rate = valu / (avg_ms * 1e-3)
        roof["limiter"] = {"bound": "valu", "achieved": round(rate / 1e9, 1),
                           "peak": round(VALU_PEAK_WAVE_INSTR_PER_S / 1e9, 1),
                           "unit": "G wave-instructions/s",
                           "frac": round(rate / VALU_PEAK_WAVE_INSTR_PER_S, 4),
                           "valu_per_launch": valu}
    else:
        roof["limiter"] = None


def optimise_leg(args, w, prec_name: str, copy_gbs: float):
    """The optimisation loop on workload w; returns the result dict."""
    import numpy as np
    import torch

    from paper_1303_0107_amd import lbm

    types = w.types()
    N = types.size
    nns = int(np.count_nonzero(types))
    prec = {"f64": lbm.LBM_F64, "f32": lbm.LBM_F32, "f16": lbm.LBM_F32_S_F16,
            "bf16": lbm.LBM_F32_S_BF16}[prec_name]
    s_bytes = {"f64": 8, "f32": 4, "f16": 2, "bf16": 2}[prec_name]
    arith = "f64" if prec_name == "f64" else "f32"
    frac = w.extra.get("frac", 0.01)
    k = 100
    print(f"# workload {w.name} {w.nx}x{w.ny} non-solid {nns} precision {prec_name}",
          file=sys.stderr, flush=True)
    lat = lbm.Lattice(types, w.tau, w.u_peak, precision=prec)
    t0 = time.perf_counter()
    settle_cap = args.settle_cap if args.settle_cap is not None else w.extra.get("cap0", 500000)
    rc, settle_steps, res = lat.run(settle_cap, args.tol, k)
    print(f"# settle: rc={rc} steps={settle_steps} r={res:.3e} "
          f"({time.perf_counter() - t0:.1f} s)", file=sys.stderr, flush=True)
    shape, tune_ms = lat.autotune(max(args.tune_steps, 800))
    rows, halo, tw, th = lbm.lbm_tb_variant_info(prec, shape)
    print(f"# autotune: shape {shape} ({rows} rows, halo {halo}); us/step "
          + " ".join(f"{x * 1e3:.3f}" for x in tune_ms), file=sys.stderr, flush=True)

    ex_ms, stats_ms = [], []

    def one_step(seed):
        t = time.perf_counter()
        r, _, _ = lat.shape_update(frac=frac, seed=seed)
        ex_ms.append((time.perf_counter() - t) * 1e3)
        rc, n, res = lat.run(args.cap, args.tol, k)
        t = time.perf_counter()
        flow, st = lat.stats()
        stats_ms.append((time.perf_counter() - t) * 1e3)
        return n, res, flow, st, r

    for i in range(args.warmup):
        one_step(1000 + i)
    torch.cuda.synchronize()
    del ex_ms[:], stats_ms[:]
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
    in_use = lbm.lbm_get_tb_variant(lat.h)

    mlups = N * sweeps / wall / 1e6
    bytes_per_step = 18 * s_bytes * nns + N
    steps_per_launch = timed_steps / max(launches, 1)
    bytes_per_launch = bytes_per_step * steps_per_launch
    avg_ms = sweep_ms / max(launches, 1)
    achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9
    n, res, flow, st, r = last
    spread = float((flow.max() - flow.min()) / flow.mean()) if len(flow) else 0.0
    kernel = "tb_kernel" if steps_per_launch > 1.0 else "step_kernel"
    full = MEASURED_TRAFFIC_PER_FULL_LAUNCH.get((w.name, prec_name, in_use))
    per_interval = -(-k // halo)  # launches per check interval
    traffic = round(full + 32 * nns / per_interval) if full else None
    valu = MEASURED_VALU_PER_FULL_LAUNCH.get((w.name, prec_name, in_use))
    roof = {
        "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
        "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
        "kernel": kernel + f" ({prec_name} storage, shape {in_use}: {rows}x64 region, "
                           f"{halo} steps per launch)",
        "bytes_per_step": bytes_per_step, "steps_per_launch": round(steps_per_launch, 3),
        "bytes_per_launch": round(bytes_per_launch), "launches": launches,
        "launch_timing": "HIP events on the handle's stream around the launches of every "
                         "4th check interval of the timed solves",
        "avg_launch_us": round(avg_ms * 1e3, 3),
        "copy_ceiling_GBs": round(copy_gbs, 1),
        "frac_of_copy_ceiling": round(achieved / copy_gbs, 4),
    }
    hbm_and_limiter(roof, traffic, valu, avg_ms)
    out = {
        "metric": METRIC,
        "value": round(mlups, 2),
        "unit": "MLUPS",
        "mflups": round(nns * sweeps / wall / 1e6, 2),
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
            "tau": w.tau, "u_peak": w.u_peak, "storage": prec_name, "arithmetic": arith,
            "step": f"exchange (frac {frac}) + solve to r<{args.tol:g} (cap {args.cap}, "
                    f"check every {k}) + outlet stats (means over two consecutive steps)",
            "sweeps_timed": sweeps,
            "last_dp": st.dp, "last_theta": st.theta, "last_dg": st.dg,
            "last_spread": spread, "last_residual": res,
            "last_flux_period_two": st.flow_p2,
            "tuned_shape": {"index": shape, "rows": rows, "halo": halo, "tile": [tw, th]},
            "shape_in_use": in_use,
            "tune_us_per_step": [round(x * 1e3, 3) for x in tune_ms],
            "exchange_ms_median": round(float(np.median(ex_ms)), 3),
            "stats_ms_median": round(float(np.median(stats_ms)), 3),
        },
        "roofline": roof,
    }
    lat.close()
    return out


def sweep_leg(args, w, prec_name: str, steps: int, copy_gbs: float):
    """Sweeps only (no exchange steps) on workload w after the autotuner:
    `steps` time steps with residual checks every 100, timed as above."""
    import numpy as np
    import torch

    from paper_1303_0107_amd import lbm

    types = w.types()
    N = types.size
    nns = int(np.count_nonzero(types))
    prec = {"f64": lbm.LBM_F64, "f32": lbm.LBM_F32}[prec_name]
    s_bytes = {"f64": 8, "f32": 4}[prec_name]
    lat = lbm.Lattice(types, w.tau, w.u_peak, precision=prec)
    lat.run(2000, 0.0, 100)
    shape, tune_ms = lat.autotune(400)
    rows, halo, tw, th = lbm.lbm_tb_variant_info(prec, shape)
    lat.run(1000, 0.0, 100)
    torch.cuda.synchronize()
    lat.profile_sweeps(True)
    t0 = time.perf_counter()
    lat.run(steps, 0.0, 100)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    timed_steps, launches, sweep_ms = lat.profile_sweeps(False)
    in_use = lbm.lbm_get_tb_variant(lat.h)
    lat.close()
    bytes_per_step = 18 * s_bytes * nns + N
    avg_ms = sweep_ms / max(launches, 1)
    spl = timed_steps / max(launches, 1)
    achieved = bytes_per_step * spl / (avg_ms * 1e-3) / 1e9
    full = MEASURED_TRAFFIC_PER_FULL_LAUNCH.get((w.name, prec_name, in_use))
    per_interval = -(-100 // halo)
    traffic = round(full + 32 * nns / per_interval) if full else None
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
            "kernel": f"tb_kernel ({prec_name} storage, shape {in_use}: {rows}x64 region, "
                      f"{halo} steps per launch)",
            "bytes_per_step": bytes_per_step, "avg_launch_us": round(avg_ms * 1e3, 3),
            "steps_per_launch": round(spl, 3),
            "frac_of_copy_ceiling": round(achieved / copy_gbs, 4)}
    hbm_and_limiter(roof, traffic, MEASURED_VALU_PER_FULL_LAUNCH.get((w.name, prec_name, in_use)),
                    avg_ms)
    print(f"# {w.name}: {steps} steps in {wall * 1e3:.1f} ms, shape {in_use}", file=sys.stderr,
          flush=True)
    return {"workload": w.name, "storage": prec_name, "steps": steps,
            "value": round(N * steps / wall / 1e6, 2), "unit": "MLUPS",
            "mflups": round(nns * steps / wall / 1e6, 2),
            "us_per_step": round(wall / steps * 1e6, 3), "roofline": roof}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5, help="timed optimisation iterations")
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--precision", choices=["f32", "f64", "f16", "bf16"], default="f32",
                    help="population storage (f64: double storage and arithmetic; f32: float "
                         "storage, float arithmetic; f16/bf16: 16-bit storage, float arithmetic)")
    ap.add_argument("--workload", default="distributor-1024x512-L3")
    ap.add_argument("--legs", default="main,channel,serve",
                    help="comma list: main (the workload's optimisation loop, or sweeps for a "
                         "channel), channel (1024x512 all-fluid sweeps), serve (short serving "
                         "run)")
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--cap", type=int, default=200000, help="step cap per solve")
    ap.add_argument("--settle-cap", type=int, default=None,
                    help="step cap of the untimed solve from rest (default: workload's)")
    ap.add_argument("--tune-steps", type=int, default=256,
                    help="steps per autotuner trial")
    ap.add_argument("--sweep-steps", type=int, default=20000,
                    help="timed time steps of a sweep leg")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--batch-steps", type=int, default=10000,
                    help="time steps per benchmark step of the batched workload")
    ap.add_argument("--batch-count", type=int, default=256)
    ap.add_argument("--serve-rate", type=float, default=50.0)
    ap.add_argument("--serve-seconds", type=float, default=60.0,
                    help="arrival window of the serving workload run on its own")
    ap.add_argument("--serve-leg-seconds", type=float, default=20.0,
                    help="arrival window of the serving leg of the default run")
    ap.add_argument("--hbm-budget-gb", type=float, default=32.0)
    ap.add_argument("--max-sessions", type=int, default=64)
    ap.add_argument("--quantum", type=int, default=40)
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path",
              file=sys.stderr)
        return 2

    import torch

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 1
    torch.cuda.set_device(0)
    if args.workload == BATCH_WORKLOAD:
        return bench_batch(args)
    if args.workload == SERVE_WORKLOAD:
        return bench_serve(args)
    legs = {x.strip() for x in args.legs.split(",") if x.strip()}
    w = workloads()[args.workload]
    copy_gbs = copy_ceiling()
    bad = 0
    if w.kind == "channel":
        leg = sweep_leg(args, w, args.precision, args.sweep_steps, copy_gbs)
        out = {"metric": METRIC, "value": leg["value"], "unit": "MLUPS", "mflups": leg["mflups"],
               "n_gpus": 1, "steps": 1, "warmup": 0, "ms_per_step": leg["us_per_step"] * 1e-3,
               "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
               "dtype": "f64" if args.precision == "f64" else "f32", "data": "synthetic",
               "config": {"workload": w.name, "nx": w.nx, "ny": w.ny, "storage": args.precision,
                          "step": "one time step (sweeps only)"},
               "roofline": leg["roofline"]}
    else:
        out = optimise_leg(args, w, args.precision, copy_gbs)
    if "channel" in legs and w.kind != "channel":
        from paper_1303_0107_amd import inputs as I
        out["channel"] = sweep_leg(args, I.CHANNEL_1024x512, "f32", args.sweep_steps, copy_gbs)
    if "serve" in legs:
        srv, bad = serve_leg(args, args.serve_rate, args.serve_leg_seconds)
        out["latency_ms"] = srv["config"]["latency_ms"]
        out["serving"] = {"value": srv["value"], "unit": "MLUPS", "mflups": srv["config"]["mflups"],
                          "requests": srv["config"]["requests"],
                          "arrivals": srv["config"]["arrivals"], "mix": srv["config"]["mix"],
                          "failed": srv["config"]["failed"],
                          "busy_seconds": srv["config"]["busy_seconds"],
                          "event_seconds": srv["config"]["event_seconds"],
                          "sweep_seconds": srv["config"]["sweep_seconds"],
                          "admit_seconds": srv["config"]["admit_seconds"],
                          "wall_seconds": srv["config"]["wall_seconds"]}
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(w.types(), w, args.cpu_seconds)
    print(json.dumps(out), flush=True)
    return 0 if not bad else 1


if __name__ == "__main__":
    sys.exit(main())
