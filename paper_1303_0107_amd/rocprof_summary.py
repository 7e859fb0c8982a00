"""Condense rocprofv3 CSV output into the short text summaries kept here.

usage: python -m paper_1303_0107_amd.rocprof_summary STATS_CSV [FETCH_CSV WRITE_CSV] --cmd "..." --kernel SUBSTR
           [--copy-bytes N] [--algo-bytes N] [--pmc CSV ...]

STATS_CSV is a --kernel-trace --stats *_kernel_stats.csv; FETCH_CSV/WRITE_CSV
are --pmc FETCH_SIZE / WRITE_SIZE *_counter_collection.csv files of the same
program.  The counters are scaled by what they read for the plain copy kernel
(__amd_rocclr_copyBuffer of --copy-bytes bytes, reads and writes each).
Each --pmc CSV (any other counters) adds, per matching kernel and grid size,
the mean of every counter it holds per dispatch.
"""
import argparse
import collections
import csv
import re
import subprocess


SHORT = [("lbm::OffsetCell<float, float, float>", "F32Cell"),
         ("lbm::OffsetCell<float, double, double>", "F32Cell(double arithmetic)"),
         ("lbm::OffsetCell<_Float16, float, float>", "H16Cell"),
         ("lbm::OffsetCell<__hip_bfloat16, float, float>", "BF16Cell"),
         ("lbm::f64::Cell", "F64Cell"), ("void ", ""), ("(anonymous namespace)::", ""),
         ("lbm::sweep::", ""), ("lbm::", "")]


# Mangled blocked-sweep names that c++filt leaves alone (it does not know the
# _Float16 mangling): tb_kernel / tb_batch_kernel of an offset cell.
_TB = re.compile(r"_ZN3lbm5sweep(\d+)(tb_kernel|tb_batch_kernel)INS_10OffsetCellI"
                 r"(DF16_|14__hip_bfloat16|f)ffEE((?:L[ib]\d+E)+)")
_CELL = {"DF16_": "H16Cell", "14__hip_bfloat16": "BF16Cell", "f": "F32Cell"}


def demangle(name: str) -> str:
    """The readable form of a mangled kernel name (c++filt), else the name."""
    if not name.startswith("_Z"):
        return name
    m = _TB.match(name)
    if m:
        args = []
        for kind, v in re.findall(r"L([ib])(\d+)E", m.group(4)):
            args.append(v if kind == "i" else ("true" if v == "1" else "false"))
        return f"{m.group(2)}<{_CELL[m.group(3)]}, {', '.join(args)}>"
    try:
        out = subprocess.run(["c++filt", name], capture_output=True, text=True, timeout=10)
        return out.stdout.strip() or name
    except (OSError, subprocess.SubprocessError):
        return name


def short(name: str) -> str:
    """Kernel name with the cell policy abbreviated and the argument list cut."""
    name = demangle(name)
    for a, b in SHORT:
        name = name.replace(a, b)
    return name.split("(")[0]


def per_kernel(path, counter):
    """Mean counter value per (kernel, grid size), dispatch counts, and the
    readings of the plain copy kernel in dispatch order."""
    agg = collections.defaultdict(list)
    copies = []
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] == counter:
            v = float(r["Counter_Value"])
            agg[(r["Kernel_Name"], int(r["Grid_Size"]))].append(v)
            if "copyBuffer" in r["Kernel_Name"]:
                copies.append((int(r["Dispatch_Id"]), v))
    copies = [v for _, v in sorted(copies)]
    return ({k: sum(v) / len(v) for k, v in agg.items()}, {k: len(v) for k, v in agg.items()},
            copies)


def copy_readings(fetch_copies, write_copies, nbytes):
    """FETCH_SIZE and WRITE_SIZE of the calibration copy of nbytes.  The two
    runs make the same copies in the same order; WRITE_SIZE of a copy reads
    the bytes it writes (in KiB), so the calibration copy is the one whose
    write reading is nbytes / 1024.  Without such a reading (or if the runs
    made different numbers of copies), the largest copy is taken."""
    if len(fetch_copies) == len(write_copies):
        for f, w in zip(fetch_copies, write_copies):
            if w * 1024.0 == nbytes:
                return f, w
    return max(fetch_copies), max(write_copies)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("stats")
    ap.add_argument("fetch", nargs="?")
    ap.add_argument("write", nargs="?")
    ap.add_argument("--cmd", required=True)
    ap.add_argument("--pmc-cmd", default="")
    ap.add_argument("--kernel", required=True)
    ap.add_argument("--copy-bytes", type=int, default=1 << 28)
    ap.add_argument("--algo-bytes", type=int, default=0)
    ap.add_argument("--pmc", action="append", default=[])
    ap.add_argument("--trace", default="",
                    help="a --kernel-trace *_kernel_trace.csv: mean duration per kernel and grid")
    a = ap.parse_args()
    print(f"command: {a.cmd}")
    print()
    print(f"{'kernel':72s} {'calls':>8s} {'avg_us':>9s} {'total_ms':>10s} {'pct':>6s}")
    for r in csv.DictReader(open(a.stats)):
        print(f"{short(r['Name'])[:72]:72s} {int(r['Calls']):8d} {float(r['AverageNs']) / 1e3:9.3f} "
              f"{float(r['TotalDurationNs']) / 1e6:10.2f} {float(r['Percentage']):6.2f}")
    if a.trace:
        print()
        print(f"mean duration per dispatch, by kernel and grid (threads), from {a.trace.split('/')[-1]}:")
        agg = collections.defaultdict(list)
        for r in csv.DictReader(open(a.trace)):
            if a.kernel in r["Kernel_Name"] or a.kernel == "*":
                g = int(r["Grid_Size_X"]) * int(r["Grid_Size_Y"]) * int(r["Grid_Size_Z"]) \
                    if "Grid_Size_X" in r else int(r["Grid_Size"])
                agg[(short(r["Kernel_Name"]), g)].append(
                    (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
        for (k, g), v in sorted(agg.items()):
            print(f"{k[:60]:60s} grid {g:>10d} dispatches {len(v):5d} mean {sum(v) / len(v):9.3f} us")
    for path in a.pmc:
        print()
        print(f"counters per dispatch (mean) from {path.split('/')[-1]}:")
        agg = collections.defaultdict(lambda: collections.defaultdict(list))
        for r in csv.DictReader(open(path)):
            if a.kernel in r["Kernel_Name"]:
                agg[(r["Kernel_Name"], int(r["Grid_Size"]))][r["Counter_Name"]].append(
                    float(r["Counter_Value"]))
        for (k, g), cs in sorted(agg.items(), key=lambda kv: -len(next(iter(kv[1].values())))):
            n = len(next(iter(cs.values())))
            vals = ", ".join(f"{c} {sum(v) / len(v):.4g}" for c, v in sorted(cs.items()))
            print(f"{short(k)[:72]} grid {g} ({n} dispatches): {vals}")
    if not a.fetch:
        return
    print()
    print(f"counters: {a.pmc_cmd}")
    fetch, nf, copies_f = per_kernel(a.fetch, "FETCH_SIZE")
    write, nw, copies_w = per_kernel(a.write, "WRITE_SIZE")
    copy_f, copy_w = copy_readings(copies_f, copies_w, a.copy_bytes)
    kib = 1024.0
    sf = a.copy_bytes / (copy_f * kib)
    sw = a.copy_bytes / (copy_w * kib)
    print(f"plain copy of {a.copy_bytes} B: FETCH_SIZE {copy_f:.1f} KiB, WRITE_SIZE {copy_w:.1f} KiB"
          f" -> scale fetch x{sf:.3f}, write x{sw:.3f}")
    for (k, g), v in sorted(fetch.items(), key=lambda kv: -kv[1]):
        if a.kernel in k:
            w = write.get((k, g), 0.0)
            fb, wb = v * kib * sf, w * kib * sw
            line = (f"{short(k)[:72]} grid {g}: dispatches {nf[(k, g)]}, fetch {fb / 1e6:.3f} MB, "
                    f"write {wb / 1e6:.3f} MB, traffic {(fb + wb) / 1e6:.3f} MB per dispatch")
            if a.algo_bytes:
                line += f" ({(fb + wb) / a.algo_bytes:.3f} x algorithmic {a.algo_bytes / 1e6:.3f} MB)"
            print(line)


if __name__ == "__main__":
    main()
