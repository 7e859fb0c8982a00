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


FIT_DRIVER = r"""
#include <cstdio>
#include <cstdlib>
#include "lbm_tiles.h"
// argv: tuned, then triples (ms, resident, tiles) per shape; prints the shape
// chosen and the shapes whose tile counts were asked for.
int main(int argc, char **argv) {
    const int tuned = std::atoi(argv[1]);
    std::vector<double> ms;
    std::vector<size_t> res, tiles;
    for (int a = 2; a + 2 < argc; a += 3) {
        ms.push_back(std::atof(argv[a]));
        res.push_back(std::strtoul(argv[a + 1], nullptr, 10));
        tiles.push_back(std::strtoul(argv[a + 2], nullptr, 10));
    }
    std::vector<int> asked;
    const int v = lbm::fitted_shape(tuned, ms, res, [&](int s) {
        asked.push_back(s);
        return tiles[s];
    });
    std::printf("%d", v);
    for (int s : asked) std::printf(" %d", s);
    std::printf("\n");
    return 0;
}
"""


@pytest.fixture(scope="module")
def fitter(tmp_path_factory):
    cxx = shutil.which("g++")
    if cxx is None:
        pytest.skip("no host C++ compiler")
    d = tmp_path_factory.mktemp("fit")
    src = d / "fit.cpp"
    src.write_text(FIT_DRIVER)
    exe = d / "fit"
    subprocess.run([cxx, "-std=c++17", "-O1", "-I", CSRC, str(src), "-o", str(exe)], check=True)

    def fit(tuned, shapes):
        argv = [str(exe), str(tuned)]
        for ms, res, tiles in shapes:
            argv += [repr(ms), str(res), str(tiles)]
        out = subprocess.run(argv, check=True, capture_output=True, text=True).stdout.split()
        return int(out[0]), [int(x) for x in out[1:]]
    return fit


# 256 CUs: one workgroup of the large shapes per CU (256 resident), two of
# the small ones (512)
SHAPES = [(2.04, 256, 236), (1.63, 256, 234), (2.59, 256, 130), (2.05, 512, 470),
          (1.98, 512, 470), (1.57, 256, 236)]


def test_tuned_shape_kept_while_it_fits(fitter):
    v, asked = fitter(5, SHAPES)
    assert v == 5 and asked == [5]


def test_fastest_fitting_shape_when_the_tuned_one_overflows(fitter):
    shapes = list(SHAPES)
    shapes[5] = (1.57, 256, 252 + 20)   # the 9-step shape now needs two rounds
    v, asked = fitter(5, shapes)
    assert v == 1                        # next fastest (1.63) that fits
    assert asked[0] == 5 and asked[1] == 1
    shapes[1] = (1.63, 256, 300)         # that one overflows too
    v, _ = fitter(5, shapes)
    assert v == 4                        # 1.98, two workgroups per CU


def test_tuned_shape_taken_back_and_none_fitting(fitter):
    # the tuned shape fits again: it is chosen whatever ran before
    assert fitter(5, SHAPES)[0] == 5
    # nothing fits: stay with the tuned shape
    shapes = [(ms, res, 10 ** 6) for ms, res, _ in SHAPES]
    assert fitter(5, shapes)[0] == 5
    # no timings: the tuned shape is returned unchanged
    assert fitter(2, [])[0] == 2
