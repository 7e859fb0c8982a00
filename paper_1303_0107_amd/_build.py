"""Compile the HIP library liblbm.so for gfx950 (in-tree)."""
from __future__ import annotations

import concurrent.futures
import os
import subprocess
import tempfile

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "liblbm.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

COMMON = [
    "-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC",
    # keep the compiler from emitting packed FP32 arithmetic
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
    # the leading pointer and integer arguments of each kernel (up to three)
    # arrive preloaded in scalar registers instead of being loaded at its start
    "-mllvm", "-amdgpu-kernarg-preload-count=3",
]
# Per source: extra flags.  The double-precision sweep and the host
# arithmetic of the reductions must not fuse multiply-adds (each IEEE
# operation rounds once, in the order written).
SOURCES = {
    "lbm_kernels.hip": [],
    "lbm_f64.hip": ["-ffp-contract=off"],
    "lbm_api.hip": ["-ffp-contract=off"],
    "lbm_serve.hip": [],
    "lbm_select.hip": [],
}


def build(verbose: bool = False, out: str = LIB, defines=()) -> str:
    inc = ["-I", os.path.join(ROOT, "include"), "-I", CSRC]
    with tempfile.TemporaryDirectory() as tmp:
        jobs = []
        for src, extra in SOURCES.items():
            obj = os.path.join(tmp, src + ".o")
            cmd = [HIPCC, *COMMON, *extra, *[f"-D{d}" for d in defines], *inc, "-c",
                   os.path.join(CSRC, src), "-o", obj]
            if verbose:
                print(" ".join(cmd), flush=True)
            jobs.append((src, obj, cmd))
        # one compiler process per source, at most four at a time
        with concurrent.futures.ThreadPoolExecutor(max_workers=4) as pool:
            results = list(pool.map(
                lambda j: subprocess.run(j[2], capture_output=True, text=True), jobs))
        for (src, _, _), res in zip(jobs, results):
            if res.returncode != 0:
                raise RuntimeError(f"hipcc failed on {src}:\n" + res.stdout + res.stderr)
        objs = [obj for _, obj, _ in jobs]
        tmp_lib = out + ".tmp"
        cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp_lib, *objs]
        res = subprocess.run(cmd, capture_output=True, text=True)
        if res.returncode != 0:
            raise RuntimeError("link failed:\n" + res.stdout + res.stderr)
        os.replace(tmp_lib, out)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
