// The inlet-and-outlets task of the boundary sums (Sec. 2.3 step 5, Eqs.
// 9-11; the pressure drop of Eq. 4), shared by the storage forms.
//
// One workgroup of kBoundaryThreads threads sums, each as a running sum in
// increasing y (the order of a sequential loop over the rows): the density
// over every outlet cell of column nx - 1, and the x momentum and the
// density over the inlet cells of column 0, with the two cell counts.  The
// threads first take up to kBoundarySpan rows (kBoundaryRowsPerThread each)
// and leave each row's values in LDS; thread 0 then adds them up in row
// order, with selects instead of branches so that the additions follow each
// other closely.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lbm_internal.h"

namespace lbm {

constexpr int kBoundaryThreads = 256, kBoundaryRowsPerThread = 4,
              kBoundarySpan = kBoundaryThreads * kBoundaryRowsPerThread;

// at(n, rho, jx): density and x momentum of the cell at pitched index n.
// o: [flow_in, rho_in, count_in, count_out, rho_out] (valid in thread 0).
template <class At>
__device__ __forceinline__ void boundary_ends(const uint16_t *cell, int nx, int ny, int pitch,
                                              At at, double (&o)[5]) {
    __shared__ double s_ro[kBoundarySpan], s_ri[kBoundarySpan], s_ji[kBoundarySpan];
    __shared__ uint8_t s_kind[kBoundarySpan];  // bit 0: outlet cell, bit 1: inlet cell
    const int t = threadIdx.x;
    double fl = 0.0, rin = 0.0, cin = 0.0, cout = 0.0, rout = 0.0;
    for (int c0 = 0; c0 < ny; c0 += kBoundarySpan) {
        // The cell words of all of a thread's rows first, then the
        // populations of all of them at once: rows that hold no boundary
        // cell (and rows past the end) read cell 0 instead, which every lane
        // shares, so that no branch separates the loads and no other cache
        // line is touched; their values are dropped by the selects.
        bool out[kBoundaryRowsPerThread], in[kBoundaryRowsPerThread];
#pragma unroll
        for (int q = 0; q < kBoundaryRowsPerThread; ++q) {
            const int y = c0 + q * kBoundaryThreads + t;
            const size_t n0 = (size_t)min(y, ny - 1) * pitch;
            const uint32_t wo = cell[n0 + nx - 1], wi = cell[n0];
            out[q] = (y < ny) & (cell_type(wo) == kOutlet);
            in[q] = (y < ny) & (cell_type(wi) == kInlet);
        }
#pragma unroll
        for (int q = 0; q < kBoundaryRowsPerThread; ++q) {
            const int r = q * kBoundaryThreads + t;
            const size_t n0 = (size_t)(c0 + r) * pitch;
            double ro, jo, ri, ji;
            at(out[q] ? n0 + nx - 1 : 0, ro, jo);
            at(in[q] ? n0 : 0, ri, ji);
            s_ro[r] = out[q] ? ro : 0.0;
            s_ri[r] = in[q] ? ri : 0.0;
            s_ji[r] = in[q] ? ji : 0.0;
            s_kind[r] = (uint8_t)((out[q] ? 1 : 0) | (in[q] ? 2 : 0));
        }
        __syncthreads();
        if (t == 0) {
            const int m = min(kBoundarySpan, ny - c0);
#pragma unroll 8
            for (int r = 0; r < m; ++r) {
                const int kd = s_kind[r];
                const bool out = (kd & 1) != 0, in = (kd & 2) != 0;
                const double a = rout + s_ro[r], b = fl + s_ji[r], c = rin + s_ri[r];
                rout = out ? a : rout;
                cout = out ? cout + 1.0 : cout;
                fl = in ? b : fl;
                rin = in ? c : rin;
                cin = in ? cin + 1.0 : cin;
            }
        }
        __syncthreads();
    }
    o[0] = fl;
    o[1] = rin;
    o[2] = cin;
    o[3] = cout;
    o[4] = rout;
}

}  // namespace lbm
