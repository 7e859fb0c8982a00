"""The paper's own run (Sec. 3.3) as a workload: a collector computed on half
its domain, W_in = 11, W_out = 52, nu = 0.04, u_in = 0.08, Re_in = 22.

The map is synthetic (the paper's figures are not available); its channel
widths follow Eq. 8 from the finest channel, and the trunk width that chain
produces is the W_out the paper states, which pins the geometric reading.
The oracle's run on it is a finding, not a pass/fail of the method: at these
numbers the merged channels carry mean speeds of 0.2-0.27 lattice units, and
BGK goes unstable (the oracle reports it instead of running on NaNs)."""
import numpy as np
import pytest

from paper_1303_0107_amd import inputs as I

W = I.PAPER_COLLECTOR_360x180


def _runs(col):
    """(start, length) of the runs of True in a boolean column."""
    out, start = [], None
    for y, v in enumerate(list(col) + [False]):
        if v and start is None:
            start = y
        elif not v and start is not None:
            out.append((start, y - start))
            start = None
    return out


def test_widths_follow_eq8_from_the_finest_channel():
    chain = I.width_law_chain(55.0, 11.0, 4)  # depth 10 mm = 55 cells at 11 cells per 2 mm
    assert round(chain[0]) == W.extra["w_out"] == 52
    # the same chain in mm is Table 1's widths (2.00, 2.91, 4.27, 6.35)
    assert [c * 2.0 / 11.0 for c in chain[1:]] == pytest.approx([6.35, 4.27, 2.91, 2.00], rel=0.01)
    assert I.paper_collector_widths() == W.widths == [52, 34, 24, 15, 11]


def test_mirror_widths_parity():
    # ny = 360: level-k centres fall on row boundaries for k <= 2 (even widths)
    assert I.mirror_widths([52.4, 34.7, 23.4, 15.9, 11.0], 360) == [52, 34, 24, 15, 11]
    assert I.mirror_widths([9.0, 9.0], 64) == [8, 8]
    # ny = 6: the level-0 centre (row 3) is a row boundary, the level-1
    # centres (1.5, 4.5) are not; ties go to the smaller width
    assert I.mirror_widths([3.0, 2.4], 6) == [2, 3]


def test_map_is_the_lower_half_of_a_sixteen_inlet_collector():
    t = W.types()
    assert t.shape == (180, 360)
    full = I.collector(360, 360, 4, W.widths)
    assert np.array_equal(np.vstack([t, t[::-1]]), full)
    inlets = _runs(t[:, 0] == I.INLET)
    assert len(inlets) == 8 and all(n == W.extra["w_in"] for _, n in inlets)
    outlets = _runs(t[:, -1] == I.OUTLET)
    assert outlets == [(180 - 26, 26)]  # half of W_out, against the symmetry line


def test_parameters():
    nu = W.extra["nu"]
    assert W.tau == pytest.approx(3 * nu + 0.5)
    assert W.u_peak == pytest.approx(1.5 * W.extra["u_in"])  # a parabola's mean is 2/3 of its peak
    assert I.reynolds_inlet(W.extra["w_in"], W.extra["u_in"], nu) == pytest.approx(22.0)


def test_oracle_reports_the_instability(orc):
    """Velocity inlets with the velocity-imposing Neumann outlet fix no density
    level: inflow exceeds outflow while the trunk speeds up, the mean density
    rises, and the run ends with EUNSTABLE (at step 3500 with checks every 100)."""
    t = W.types()
    lat = orc.Lattice(t, W.tau, W.u_peak, flags=W.extra["flags"])
    status, steps, _ = lat.run(1000, 0.0, 100)
    assert status == orc.OK and steps == 1000
    rho, ux, uy = lat.macro()
    assert rho[t != 0].mean() > 1.3
    s = lat.outlet_stats()
    assert s.flow_in > 2 * s.flow.sum() > 0
    status, steps, _ = lat.run(5000, 0.0, 100)
    assert status == orc.EUNSTABLE and 1000 + steps == 3500


def test_mirror_widths_give_mirror_symmetric_maps():
    rng = np.random.default_rng(0)
    checked = 0
    for _ in range(60):
        ny = int(rng.integers(40, 200))
        L = int(rng.integers(1, 4))
        ws = I.mirror_widths(list(rng.uniform(2.5, ny / 2 ** (L + 1), L + 1)), ny)
        if min(ws) < 2 or ny // 2 ** L < ws[-1] + 2:
            continue
        t = I.distributor(96, ny, L, ws)
        assert np.array_equal(t, t[::-1]), (ny, L, ws)
        checked += 1
    assert checked >= 20
