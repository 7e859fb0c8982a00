"""The allocation-free statistics entry point against the allocating one,
through the C ABI: identical results on two calls in a row (the second on a
smaller lattice, so the shared scratch holds the first call's larger data),
the state left unchanged, and the limits refused with an error."""
import ctypes

import numpy as np
import pytest

from paper_1303_0107_amd import inputs as I
from paper_1303_0107_amd import lbm

pytestmark = pytest.mark.gpu

FIELDS = ("n_outlets", "n_fluid", "n_nonsolid", "flow_in", "dp", "theta", "dg", "flow_ave",
          "mass", "residual", "steps", "flow_p2")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    lbm.load()


def _same(a, b):
    for f in FIELDS:
        x, y = getattr(a, f), getattr(b, f)
        assert x == y or (np.isnan(x) and np.isnan(y)), f


@pytest.mark.parametrize("prec", [lbm.LBM_F64, lbm.LBM_F32])
def test_noalloc_stats_equal_the_allocating_call(prec):
    cases = [(I.HEADLINE_1024x512, 900), (I.CORRECTNESS_128x64, 400)]
    for wl, steps in cases:  # the second lattice is the smaller one
        print(f"noalloc stats: {wl.name} prec={prec}", flush=True)
        g = lbm.Lattice(wl.types(), wl.tau, wl.u_peak, precision=prec)
        g.run(steps, 0.0, 100)
        before = g.state()
        fa, sa = lbm.lbm_outlet_stats_noalloc(g.h)
        fb, sb = lbm.lbm_outlet_stats(g.h)
        assert np.array_equal(fa, fb)
        _same(sa, sb)
        assert np.array_equal(g.state(), before)
        fc, sc = lbm.lbm_outlet_stats_noalloc(g.h)  # repeated: same bits
        assert np.array_equal(fa, fc)
        _same(sa, sc)
        g.close()


def test_noalloc_limits_are_refused():
    """1050 outlets exceed the entry point's 1024; the allocating call still
    serves the lattice."""
    ny, nx = 2104, 64
    t = I.channel(nx, ny)
    t[2:-2:2, -1] = 0  # every other row of the outlet column closed
    g = lbm.Lattice(t, 0.7, 0.02, precision=lbm.LBM_F32)
    flow, s = lbm.lbm_outlet_stats(g.h, flow_cap=2048)
    assert s.n_outlets > 1024
    with pytest.raises(lbm.LbmError, match="outlets"):
        lbm.lbm_outlet_stats_noalloc(g.h, flow_cap=2048)
    g.close()
