// Launch order of the temporally blocked sweep's tiles (host code only).
#pragma once

#include <stddef.h>
#include <stdint.h>

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

}  // namespace lbm
