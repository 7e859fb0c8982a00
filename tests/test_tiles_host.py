"""The blocked sweep's launch order (host code, csrc/lbm_tiles.h), compiled
with the host C++ compiler: every tile is launched exactly once, and the
tiles workgroup slots g = 8j + k give XCD k are its runs of the row-major
list, in order."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1303_0107_amd", "csrc")

DRIVER = r"""
#include <cstdio>
#include <cstdlib>
#include "lbm_tiles.h"
int main(int argc, char **argv) {
    const size_t n = std::strtoul(argv[1], nullptr, 10), runs = std::strtoul(argv[2], nullptr, 10);
    std::vector<int32_t> list(n);
    for (size_t i = 0; i < n; ++i) list[i] = (int32_t)i;
    for (int32_t v : lbm::dealt_tiles(list, runs)) std::printf("%d\n", v);
    return 0;
}
"""


@pytest.fixture(scope="module")
def dealer(tmp_path_factory):
    cxx = shutil.which("g++")
    if cxx is None:
        pytest.skip("no host C++ compiler")
    d = tmp_path_factory.mktemp("tiles")
    src = d / "deal.cpp"
    src.write_text(DRIVER)
    exe = d / "deal"
    subprocess.run([cxx, "-std=c++17", "-O1", "-I", CSRC, str(src), "-o", str(exe)], check=True)

    def deal(n, runs):
        out = subprocess.run([str(exe), str(n), str(runs)], check=True, capture_output=True,
                             text=True).stdout.split()
        return [int(v) for v in out]
    return deal


def expected_runs(n, runs):
    """XCD k's tiles: runs k, k + 8, ... of the list cut into `runs` pieces
    whose sizes differ by at most one (the longer ones first)."""
    base, extra = divmod(n, runs)
    pieces, at = [], 0
    for r in range(runs):
        size = base + (1 if r < extra else 0)
        pieces.append(list(range(at, at + size)))
        at += size
    return [sum((pieces[r] for r in range(k, runs, 8)), []) for k in range(8)]


@pytest.mark.parametrize("runs", [8, 16, 32])
@pytest.mark.parametrize("n", [0, 1, 7, 8, 9, 31, 32, 33, 234, 236, 252, 257, 1216, 18944])
def test_every_tile_once_and_runs_per_xcd(dealer, n, runs):
    out = dealer(n, runs)
    assert sorted(out) == list(range(n))
    want = expected_runs(n, runs)
    for k in range(8):
        assert out[k::8] == want[k]
