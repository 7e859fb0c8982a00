// Launch order of the temporally blocked sweep's tiles (host code only).
#pragma once

#include <stddef.h>
#include <stdint.h>

#include <algorithm>
#include <vector>

namespace lbm {

// Workgroup g of a launch runs on XCD g mod 8, and each XCD has its own L2.
// The row-major tile list is cut into `runs` contiguous runs (a multiple of
// 8, sizes differing by at most one) and XCD k takes runs k, k + 8, ...:
// tiles whose regions overlap (the halo cells) then mostly read them through
// the same L2.  Measured: one run per XCD (bands of tile rows) is fastest
// for the two-copy bodies; the in-place body is fastest with 32 runs, its
// densest tiles spread over the XCDs.
inline std::vector<int32_t> dealt_tiles(const std::vector<int32_t> &list, size_t runs) {
    const size_t n = list.size(), rb = n / runs, re = n % runs;
    std::vector<std::vector<int32_t>> xcd(8);
    size_t at = 0;
    for (size_t r = 0; r < runs; ++r) {
        const size_t len = rb + (r < re ? 1 : 0);
        xcd[r % 8].insert(xcd[r % 8].end(), list.begin() + at, list.begin() + at + len);
        at += len;
    }
    // XCD sizes differ by at most one, the larger ones first: slots 8j + k
    // cover [0, n) exactly
    std::vector<int32_t> out(n);
    for (size_t k = 0; k < 8; ++k)
        for (size_t j = 0; j < xcd[k].size(); ++j) out[8 * j + k] = xcd[k][j];
    return out;
}

// Region shape to run after the mask has changed.  The autotuner's timings
// (ms[v] per step for shape v) hold while a shape's active tiles all run in
// one round of workgroups: tiles(v) <= resident[v], the workgroups of shape v
// the chip holds at once (CUs x workgroups per CU by LDS).  The tuned shape is
// kept (or taken back) whenever it fits; otherwise the fastest timed shape
// that fits; the tuned shape when none does.  tiles(v) is called only for
// shapes that are considered, in order of their timings.
template <typename TileCount>
int fitted_shape(int tuned, const std::vector<double> &ms,
                 const std::vector<size_t> &resident, TileCount tiles) {
    const int nv = (int)ms.size();
    if (tuned < 0 || tuned >= nv || (int)resident.size() != nv) return tuned;
    if (tiles(tuned) <= resident[tuned]) return tuned;
    std::vector<int> order(nv);
    for (int v = 0; v < nv; ++v) order[v] = v;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return ms[a] < ms[b]; });
    for (int v : order)
        if (v != tuned && tiles(v) <= resident[v]) return v;
    return tuned;
}

}  // namespace lbm
