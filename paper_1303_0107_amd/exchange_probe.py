"""Time the exchange step (Sec. 2.2-2.3 steps 3-4) on three distributor sizes.

python -m paper_1303_0107_amd.exchange_probe   (or run the file; needs the GPU)

For 1024x512 (L3), 2048x1024 and 4096x2048 (L4) distributors at tau 0.7,
u_peak 0.04, FP32 storage: 300 steps from rest, then 14 exchange steps
(frac 0.01, seeds 0..13) with 40 steps between them; prints the candidate
counts, K_eff and the median host wall time of lbm_shape_update over the
last 12.  Used for the exchange-step profile kept with the sources.
"""
import os
import sys
import time

import numpy as np

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))


def main():
    import torch

    from paper_1303_0107_amd import inputs as I, lbm
    torch.cuda.set_device(0)
    for nx, L in ((1024, 3), (2048, 4), (4096, 4)):
        ny = nx // 2
        g = lbm.Lattice(I.distributor(nx, ny, L), 0.7, 0.04, precision=lbm.LBM_F32)
        g.run(300, 0.0, 100)
        ts = []
        for it in range(14):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r, _, _ = g.shape_update(frac=0.01, seed=it)
            ts.append(time.perf_counter() - t0)
            g.run(40, 0.0, 40)
        ts = np.array(ts[2:]) * 1e3
        print(f"{nx}x{ny}: candidates {r.n_cand_fluid}/{r.n_cand_solid} k_eff {r.k_eff} "
              f"exchange ms median {np.median(ts):.3f} min {ts.min():.3f}", flush=True)
        g.close()


if __name__ == "__main__":
    main()
