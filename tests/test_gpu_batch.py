"""Region shapes, the autotuner and batched sweeps, through the C ABI.

Each of these only changes how the time steps are scheduled on the chip, so
the first bar is bit-identity with the plain path: one lattice on its own,
one launch per step.  Batch members are also compared with the FP64 oracle
directly: bit for bit in double precision, within 1e-5 in single."""
import numpy as np
import pytest

import oracle
from paper_1303_0107_amd import inputs as I
from paper_1303_0107_amd import lbm
from parity_helpers import fields_ok

pytestmark = pytest.mark.gpu

PRECS = [lbm.LBM_F64, lbm.LBM_F32, lbm.LBM_F32_S_F16, lbm.LBM_F32_S_BF16]
GRAPH_LAUNCHES = 16  # launches per captured batch graph


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    lbm.load()


def _obstacle_channel(nx, ny, seed):
    t = I.channel(nx, ny)
    rng = np.random.default_rng(seed)
    inner = t[2:-2, 3:-3]
    inner[rng.random(inner.shape) < 0.1] = 0
    return t


def _members(n, prec):
    """n uneven distributor candidates (sizes, levels, widths, tau, u_peak)."""
    cands = I.batch_candidates(count=n, seed=11)
    return cands, [lbm.Lattice(c.types(), c.tau, c.u_peak, precision=prec) for c in cands]


def _batch_variants(prec):
    """Region shapes, then the single-step mode."""
    return range(lbm.lbm_tb_variant_count(prec) + 1)


def _steps_per_launch(prec, variant):
    if variant == lbm.lbm_tb_variant_count(prec):
        return 1
    return lbm.lbm_tb_variant_info(prec, variant)[1]


def _steps_covering_graph_eager_and_tail(prec, variant=0):
    halo = _steps_per_launch(prec, variant)
    return GRAPH_LAUNCHES * halo + 3 * halo + 5


@pytest.mark.parametrize("prec", PRECS)
def test_every_region_shape_matches_single_steps(prec, monkeypatch):
    t = _obstacle_channel(190, 75, 5)
    res = []
    variants = range(lbm.lbm_tb_variant_count(prec))
    for v in [None, *variants]:
        monkeypatch.setenv("LBM_TB", "0" if v is None else "1")
        g = lbm.Lattice(t, 0.65, 0.05, precision=prec)
        if v is not None:
            g.set_tb_variant(v)
        out = []
        g.run(203, 0.0, 41)
        out.append(g.state())
        g.shape_update(frac=0.02, seed=4)
        g.run(99, 0.0, 99)
        out += [g.state(), g.mask()]
        res.append(out)
        g.close()
    for v, out in zip(variants, res[1:]):
        for x, y in zip(res[0], out):
            assert np.array_equal(x, y), f"shape {v}"


@pytest.mark.parametrize("prec", [lbm.LBM_F64, lbm.LBM_F32])
def test_autotune_leaves_no_trace(prec):
    t = _obstacle_channel(300, 90, 6)
    a = lbm.Lattice(t, 0.7, 0.04, precision=prec)
    b = lbm.Lattice(t, 0.7, 0.04, precision=prec)
    for g in (a, b):
        g.run(150, 0.0, 50)
    before = a.state()
    steps_before = a.stats()[1].steps
    res_before = a.stats()[1].residual
    best, ms = a.autotune(60)
    assert 0 <= best < lbm.lbm_tb_variant_count(prec)
    assert np.all(np.isfinite(ms)) and np.all(ms > 0)
    assert ms[best] == ms.min()
    assert np.array_equal(a.state(), before)
    assert a.stats()[1].steps == steps_before
    assert a.stats()[1].residual == res_before
    for g in (a, b):
        g.run(230, 0.0, 23)
    assert np.array_equal(a.state(), b.state())


@pytest.mark.parametrize("single_step", [False, True])
@pytest.mark.parametrize("prec", PRECS)
def test_batch_matches_each_lattice_alone(prec, single_step):
    """Uneven candidates (sizes, levels, widths, tau, inlet peak) advanced in
    one batch equal each lattice advanced alone, bit for bit, over runs that
    use the captured graph, eager launches and a short last launch, and over
    a second run that starts on the other buffer."""
    cands, batch_m = _members(7, prec)
    alone = [lbm.Lattice(c.types(), c.tau, c.u_peak, precision=prec) for c in cands]
    bt = lbm.Batch(batch_m)
    v = lbm.lbm_tb_variant_count(prec) if single_step else 0
    bt.configure(v, 0)
    items, spl, cells = bt.info()
    assert spl == _steps_per_launch(prec, v)
    assert cells == sum(int(np.count_nonzero(c.types())) for c in cands)
    assert items > 0
    s1 = _steps_covering_graph_eager_and_tail(prec, v)
    s2 = 2 * spl + 1
    for s in (s1, s2):
        ms = bt.run(s)
        assert ms > 0
        for g in alone:
            g.run(s, 0.0, s)
        for k, (x, y) in enumerate(zip(batch_m, alone)):
            assert np.array_equal(x.state(), y.state()), f"member {k} after {s} steps"
            assert x.stats()[1].steps == y.stats()[1].steps
    if prec in (lbm.LBM_F64, lbm.LBM_F32):
        # three members against the oracle run the same number of steps
        for k in range(3):
            c, g = cands[k], batch_m[k]
            o = oracle.Lattice(c.types(), c.tau, c.u_peak)
            o.run(s1 + s2, 0.0, 100)
            if prec == lbm.LBM_F64:
                assert np.array_equal(g.state(), o.fs), f"member {k} vs oracle"
            else:
                assert fields_ok(c.types(), g.macro(), o.macro(), 1e-5, f"batch member {k}")
    bt.close()


@pytest.mark.parametrize("prec", [lbm.LBM_F32, lbm.LBM_F32_S_F16])
def test_every_batch_configuration_gives_the_same_bits(prec):
    cands = I.batch_candidates(count=4, seed=12)
    steps = max(_steps_covering_graph_eager_and_tail(prec, v) for v in _batch_variants(prec))
    ref = None
    for v in _batch_variants(prec):
        for order in (0, 1):
            ms = [lbm.Lattice(c.types(), c.tau, c.u_peak, precision=prec) for c in cands]
            bt = lbm.Batch(ms)
            bt.configure(v, order)
            bt.run(steps)
            bt.run(37)
            states = [m.state() for m in ms]
            if ref is None:
                ref = states
            else:
                for k, (x, y) in enumerate(zip(ref, states)):
                    assert np.array_equal(x, y), f"shape {v} order {order} member {k}"
            bt.close()


def test_batch_tune_leaves_no_trace():
    prec = lbm.LBM_F32
    cands, ms = _members(5, prec)
    twins = [lbm.Lattice(c.types(), c.tau, c.u_peak, precision=prec) for c in cands]
    bt = lbm.Batch(ms)
    bt.run(50)
    for g in twins:
        g.run(50, 0.0, 50)
    before = [m.state() for m in ms]
    bv, bo, t = bt.tune(40)
    nv = lbm.lbm_tb_variant_count(prec) + 1
    assert 0 <= bv < nv and bo in (0, 1)
    assert t.shape == (2 * nv,) and np.all(t > 0) and t[2 * bv + bo] == t.min()
    for x, y in zip(before, ms):
        assert np.array_equal(x, y.state())
    assert all(m.stats()[1].steps == 50 for m in ms)
    bt.run(123)
    for g in twins:
        g.run(123, 0.0, 123)
    for x, y in zip(ms, twins):
        assert np.array_equal(x.state(), y.state())


def test_batch_follows_shape_updates():
    """A member's exchange step changes its tile list; the next batch run
    picks it up (new fluid cells are swept, new solid ones are not)."""
    prec = lbm.LBM_F32
    cands, ms = _members(3, prec)
    twins = [lbm.Lattice(c.types(), c.tau, c.u_peak, precision=prec) for c in cands]
    bt = lbm.Batch(ms)
    for it in range(3):
        bt.run(300)
        for g in twins:
            g.run(300, 0.0, 300)
        for k in (it % 3,):
            ra = ms[k].shape_update(frac=0.05, seed=it)[0]
            rb = twins[k].shape_update(frac=0.05, seed=it)[0]
            assert ra.k_eff == rb.k_eff > 0
    bt.run(77)
    for g in twins:
        g.run(77, 0.0, 77)
    for x, y in zip(ms, twins):
        assert np.array_equal(x.mask(), y.mask())
        assert np.array_equal(x.state(), y.state())


def test_batch_rejects_bad_requests():
    a = lbm.Lattice(I.channel(64, 16), 0.8, 0.02, precision=lbm.LBM_F32)
    b = lbm.Lattice(I.channel(64, 16), 0.8, 0.02, precision=lbm.LBM_F64)
    with pytest.raises(lbm.LbmError):
        lbm.lbm_batch_create([a.h, b.h])
    with pytest.raises(lbm.LbmError):
        lbm.lbm_batch_create([a.h, a.h])
    with pytest.raises(lbm.LbmError):
        lbm.lbm_batch_create([])
    bt = lbm.Batch([a])
    with pytest.raises(lbm.LbmError):
        bt.configure(lbm.lbm_tb_variant_count(lbm.LBM_F32) + 1, 0)
    with pytest.raises(lbm.LbmError):
        bt.configure(0, 2)
    with pytest.raises(lbm.LbmError):
        bt.run(-1)
    assert bt.run(0) >= 0
    with pytest.raises(lbm.LbmError):
        a.set_tb_variant(-1)
    bt.close()
