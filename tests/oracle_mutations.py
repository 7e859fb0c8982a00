"""Mutation check of the oracle's pins (CPU only; run by hand, not collected).

Each mutation below is a plausible mistake in the oracle (a dropped term, a
wrong sign, index or operand, a misread formula).  For each, the oracle is
copied to a temporary tree, the mistake is planted in the copy's C source,
the copy is compiled, and the CPU pin tests run against it; the pins must
fail for every mutation.  The repository's own oracle is never modified.

    python tests/oracle_mutations.py [-k SUBSTRING] [-j JOBS]

Prints one line per mutation (killed by which test, or SURVIVED) and exits
non-zero if any mutation survived.
"""
import argparse
import concurrent.futures as cf
import os
import shutil
import subprocess
import sys
import tempfile

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PIN_TESTS = ["tests/test_oracle_pins.py", "tests/test_oracle_exact_step.py",
             "tests/test_oracle_balance.py", "tests/test_oracle_shape.py",
             "tests/test_oracle_variants.py", "tests/test_paper_case.py"]

# (name, text in oracle/lbm_oracle.c, replacement, occurrence to replace (1-based))
MUTATIONS = [
    ("residual: squared ratio", "return sqrt(num) / sqrt(den);", "return num / den;", 1),
    ("residual: normalised by the previous field",
     "den += ux[n] * ux[n] + uy[n] * uy[n];", "den += pux[n] * pux[n] + puy[n] * puy[n];", 1),
    ("equilibrium: quadratic term doubled",
     "0.5 * (cu * cu) * (INV_CS2 * INV_CS2)", "(cu * cu) * (INV_CS2 * INV_CS2)", 1),
    ("equilibrium: sign of the u.u term", "0.5 * uu * INV_CS2)", "(-0.5) * uu * INV_CS2)", 1),
    ("equilibrium: linear term without 1/cs2", "1.0 + cu * INV_CS2", "1.0 + cu", 1),
    ("relaxation: rate tau instead of 1/tau", "const double omega = 1.0 / tau;",
     "const double omega = tau;", 2),
    ("relaxation: moved away from equilibrium", "fs[i * N + n] = fi - omega * (fi - feq[i]);",
     "fs[i * N + n] = fi + omega * (fi - feq[i]);", 1),
    ("streaming: push instead of pull", "int sx = x - CX[i], sy = y - CY[i]",
     "int sx = x + CX[i], sy = y + CY[i]", 1),
    ("bounce-back: same population returned", "if (wall) return fs[OPP[i] * N + n];",
     "if (wall) return fs[i * N + n];", 1),
    ("velocity set: a diagonal mislabelled", "static const int CX[Q] = {0, 1, 0, -1, 0, 1, -1, -1, 1};",
     "static const int CX[Q] = {0, 1, 0, -1, 0, 1, -1, 1, -1};", 1),
    ("weights: diagonal 1/18", "1.0 / 36.0", "1.0 / 18.0", 1),
    ("moments: y momentum from c_x", "my += CY[i] * f[i];", "my += CX[i] * f[i];", 1),
    ("inlet closure: density denominator sign", "/ (1.0 - ux);", "/ (1.0 + ux);", 1),
    ("inlet closure: transverse correction sign", "f[5 * N + n] = f7 - 0.5 * (f2 - f4)",
     "f[5 * N + n] = f7 + 0.5 * (f2 - f4)", 1),
    ("inlet closure: normal population coefficient", "f[1 * N + n] = f3 + (2.0 / 3.0) * ru;",
     "f[1 * N + n] = f3 + (1.0 / 3.0) * ru;", 1),
    ("outlet closure: velocity sign", "double ux = -1.0 + (f0 + f2 + f4 + 2.0 * (f1 + f5 + f8)) / rho_out;",
     "double ux = 1.0 - (f0 + f2 + f4 + 2.0 * (f1 + f5 + f8)) / rho_out;", 1),
    ("Neumann outlet: transverse velocity dropped", "- (1.0 / 6.0) * ru - 0.5 * rv;",
     "- (1.0 / 6.0) * ru;", 1),
    ("symmetry plane: population not mirrored", "pop = MIRY[i];", "pop = i;", 1),
    ("pressure drop: no c_s^2", "return (rin - rout) / INV_CS2;", "return (rin - rout);", 1),
    ("pressure drop: sum instead of mean",
     "double rin = cnt_in ? rho_in_sum / (double)cnt_in : 0.0;", "double rin = rho_in_sum;", 1),
    ("flow rate: density instead of momentum", "flow[nout - 1] += jx;", "flow[nout - 1] += r;", 1),
    ("theta: min over max", "*theta = mx / mn;", "*theta = mn / mx;", 1),
    ("D_g: divided by n instead of n - 1", "sqrt(d / (double)(nout - 1))", "sqrt(d / (double)nout)", 1),
    ("two-step mean: second state dropped", "flow[k] = 0.5 * (flow[k] + fb[k]);",
     "flow[k] = flow[k];", 1),
    ("mass: solid cells counted", "        if (type[n] == T_SOLID) continue;\n        for (int i = 0; i < Q; ++i) fc[i] = fs[i * N + n];\n        moments9(fc, &r, &jx, &jy);\n        m += r;",
     "        for (int i = 0; i < Q; ++i) fc[i] = fs[i * N + n];\n        moments9(fc, &r, &jx, &jy);\n        m += r;", 1),
    ("Eq. 5: normal instead of tangential speed", "double tang = DX[d] != 0 ? fabs(uy[m]) : fabs(ux[m]);",
     "double tang = DX[d] != 0 ? fabs(ux[m]) : fabs(uy[m]);", 1),
    ("Eq. 6: density dropped", "double key = criterion == CRIT_PAPER ? rho[n] * t3 : t3;",
     "double key = t3;", 1),
    ("exchange: fluid cells with the highest keys removed", "qsort(cf, nfc, sizeof(cand_t), cmp_ascending);",
     "qsort(cf, nfc, sizeof(cand_t), cmp_descending);", 1),
    ("exchange: K rounded up", "int64_t K = (int64_t)floor(frac * (double)nf);",
     "int64_t K = (int64_t)ceil(frac * (double)nf);", 1),
    ("exchange: ties by descending hash", "    if (a->hash < b->hash) return -1;\n    if (a->hash > b->hash) return 1;\n    return (a->idx > b->idx) - (a->idx < b->idx);\n}\n\nstatic int cmp_descending",
     "    if (a->hash > b->hash) return -1;\n    if (a->hash < b->hash) return 1;\n    return (a->idx > b->idx) - (a->idx < b->idx);\n}\n\nstatic int cmp_descending", 1),
    ("exchange: WARM re-initialisation leaves new fluid cells empty", "fs[i * N + cs[k].idx] = WT[i];",
     "fs[i * N + cs[k].idx] = 0.0;", 1),
    ("SplitMix64: wrong shift", "z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;",
     "z = (z ^ (z >> 31)) * 0xbf58476d1ce4e5b9ULL;", 1),
]


def plant(src: str, old: str, new: str, occurrence: int) -> str:
    pos = -1
    for _ in range(occurrence):
        pos = src.find(old, pos + 1)
        if pos < 0:
            raise ValueError(f"mutation site not found: {old[:60]!r}")
    return src[:pos] + new + src[pos + len(old):]


def run_one(mut):
    name, old, new, occ = mut
    with tempfile.TemporaryDirectory(prefix="orc_mut_") as tmp:
        for d in ("oracle", "tests", "paper_1303_0107_amd"):
            shutil.copytree(os.path.join(ROOT, d), os.path.join(tmp, d),
                            ignore=shutil.ignore_patterns("*.so", "__pycache__", "csrc", "*.tmp"))
        path = os.path.join(tmp, "oracle", "lbm_oracle.c")
        with open(path) as fh:
            src = fh.read()
        with open(path, "w") as fh:
            fh.write(plant(src, old, new, occ))
        env = dict(os.environ, OMP_NUM_THREADS="2")
        build = subprocess.run([sys.executable, "-c", "import oracle; oracle.build()"], cwd=tmp,
                               env=env, capture_output=True, text=True)
        if build.returncode != 0:
            return name, "killed by the compiler"
        r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-m", "not gpu", "-p",
                            "no:cacheprovider", *PIN_TESTS], cwd=tmp, env=env,
                           capture_output=True, text=True, timeout=1800)
        if r.returncode == 0:
            return name, "SURVIVED"
        failed = [l.split(" ")[1] for l in r.stdout.splitlines() if l.startswith("FAILED ")]
        return name, "killed by " + (failed[0] if failed else f"pytest rc {r.returncode}")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("-k", default="")
    ap.add_argument("-j", type=int, default=4)
    a = ap.parse_args()
    muts = [m for m in MUTATIONS if a.k in m[0]]
    with open(os.path.join(ROOT, "oracle", "lbm_oracle.c")) as fh:
        src = fh.read()
    for m in muts:
        plant(src, m[1], m[2], m[3])  # every site exists before anything runs
    survived = 0
    with cf.ThreadPoolExecutor(a.j) as ex:
        for name, verdict in ex.map(run_one, muts):
            survived += verdict == "SURVIVED"
            print(f"{name:60s} {verdict}", flush=True)
    print(f"{len(muts) - survived} of {len(muts)} mutations killed")
    return 1 if survived else 0


if __name__ == "__main__":
    sys.exit(main())
