"""The request server (continuous batching) through the C ABI.

Every lattice's arithmetic is independent of the others and of how its
steps are grouped into launches, so the bar is bit-identity: a request's
result (outlet statistics and the digest of its final state and mask) is
the same in a mix of concurrent requests, alone on a server, and done by
hand with the handle calls the request stands for."""
import time

import numpy as np
import pytest

import oracle
from paper_1303_0107_amd import inputs as I
from paper_1303_0107_amd import lbm
from parity_helpers import f64_state_digest

pytestmark = pytest.mark.gpu
GiB = 1 << 30


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    lbm.load()


def _requests(n, seed=21, precs=(lbm.LBM_F32, lbm.LBM_F32_S_F16)):
    rng = np.random.default_rng(seed)
    out = []
    for k, c in enumerate(I.batch_candidates(count=n, seed=seed)):
        prec = precs[k % len(precs)]
        if k % 3 == 0:
            r = lbm.make_request(c.nx, c.ny, c.levels, c.widths, c.tau, c.u_peak, prec,
                                 lbm.LBM_REQ_SOLVE, solve_steps=int(rng.integers(30, 130)))
        else:
            r = lbm.make_request(c.nx, c.ny, c.levels, c.widths, c.tau, c.u_peak, prec,
                                 lbm.LBM_REQ_OPTIMIZE, solve_steps=int(rng.integers(20, 90)),
                                 iterations=int(rng.integers(1, 4)),
                                 steps_per_iteration=int(rng.integers(10, 50)),
                                 frac=0.02, seed=100 + k)
        out.append(r)
    return out


def _by_hand(r):
    """The handle calls a request stands for."""
    g = r.geom
    lat = lbm.Lattice(None, g.tau, g.u_peak, g.rho_out, g.precision, g.nx, g.ny, g.levels,
                      list(g.widths)[:g.levels + 1])
    if r.solve_steps:
        lat.run(r.solve_steps, 0.0, r.solve_steps)
    if r.kind == lbm.LBM_REQ_OPTIMIZE:
        for it in range(r.iterations):
            p = r.shape
            lat.shape_update(p.frac, p.seed + it, p.band_x, p.band_y, p.criterion, p.reinit)
            if r.steps_per_iteration:
                lat.run(r.steps_per_iteration, 0.0, r.steps_per_iteration)
    flow, st = lat.stats()
    d = lat.digest()
    lat.close()
    return d, st


def _by_oracle(r):
    """The request's work done by the FP64 oracle: returns the oracle lattice
    and its steady statistics (two-step means)."""
    g = r.geom
    o = oracle.Lattice(I.distributor(g.nx, g.ny, g.levels, list(g.widths)[:g.levels + 1]),
                       g.tau, g.u_peak, g.rho_out)
    if r.solve_steps:
        o.run(r.solve_steps, 0.0, 100)
    if r.kind == lbm.LBM_REQ_OPTIMIZE:
        p = r.shape
        for it in range(r.iterations):
            o.shape_update(p.frac, p.seed + it, p.band_x, p.band_y, p.criterion, p.reinit)
            if r.steps_per_iteration:
                o.run(r.steps_per_iteration, 0.0, 100)
    return o, o.outlet_stats2()


def _run(server, reqs, stagger=None):
    ids = []
    for k, r in enumerate(reqs):
        ids.append(server.submit(r))
        if stagger and k % stagger == stagger - 1:
            time.sleep(0.02)
    server.drain()
    res = {x.id: x for x in server.poll(cap=len(reqs) + 8)}
    return [res[i] for i in ids]


def _same(a, b):
    assert a.status == b.status == lbm.LBM_OK
    assert a.digest == b.digest
    assert a.steps == b.steps and a.iterations_done == b.iterations_done
    for f in ("dp", "theta", "dg", "flow_in", "mass", "flow_ave"):
        x, y = getattr(a.stats, f), getattr(b.stats, f)
        assert x == y or (np.isnan(x) and np.isnan(y)), f


def test_results_are_identical_alone_and_in_the_mix():
    reqs = _requests(12)
    srv = lbm.Server(hbm_budget=64 * GiB, max_sessions=16, quantum=20)
    mix = _run(srv, reqs, stagger=3)
    st = srv.stats()
    srv.close()
    assert st.completed == len(reqs) and st.rejected == 0 and st.rounds > 0
    assert st.cell_steps == sum(x.steps * x.cells for x in mix)
    for r, m in zip(reqs, mix):
        alone_srv = lbm.Server(hbm_budget=64 * GiB, max_sessions=1, quantum=7)
        (alone,) = _run(alone_srv, [r])
        alone_srv.close()
        _same(m, alone)
        want_steps = r.solve_steps + (r.iterations * r.steps_per_iteration
                                      if r.kind == lbm.LBM_REQ_OPTIMIZE else 0)
        assert m.steps == want_steps
        assert m.t_submit <= m.t_admit <= m.t_done


def test_served_results_match_the_oracle():
    """Requests served in a mix of double, single and half-storage requests
    against the FP64 oracle doing the same work: double-precision requests
    (solve and optimise) bit for bit (the digest of the final state and mask,
    computed from the oracle's state, and every statistic); single-precision
    requests within 1e-5 on the pressure drop, inflow, mass and theta."""
    reqs = _requests(10, seed=24,
                     precs=(lbm.LBM_F64, lbm.LBM_F32, lbm.LBM_F64, lbm.LBM_F32_S_F16))
    srv = lbm.Server(hbm_budget=64 * GiB, max_sessions=16, quantum=20)
    res = _run(srv, reqs, stagger=2)
    srv.close()
    checked = {lbm.LBM_F64: set(), lbm.LBM_F32: set()}
    for r, m in zip(reqs, res):
        prec = r.geom.precision
        if prec not in checked:
            continue
        assert m.status == lbm.LBM_OK
        o, so = _by_oracle(r)
        if prec == lbm.LBM_F64:
            assert m.digest == f64_state_digest(o.types, o.fs)
            for f in ("dp", "theta", "dg", "flow_in", "flow_p2"):
                assert getattr(m.stats, f) == getattr(so, f), f
            # the mass is a block-wise sum on the device (another order)
            assert abs(m.stats.mass - so.mass) < 1e-13 * so.mass
        else:
            assert abs(m.stats.dp - so.dp) < 1e-5 * abs(so.dp)
            assert abs(m.stats.flow_in - so.flow_in) < 1e-5 * abs(so.flow_in)
            assert abs(m.stats.mass - so.mass) < 1e-5 * so.mass
            if np.abs(so.flow).min() > 1e-3 * abs(so.flow_in):  # outflow established
                assert abs(m.stats.theta - so.theta) < 1e-5
        checked[prec].add(r.kind)
    assert checked[lbm.LBM_F64] == {lbm.LBM_REQ_SOLVE, lbm.LBM_REQ_OPTIMIZE}
    assert lbm.LBM_REQ_SOLVE in checked[lbm.LBM_F32]


def test_server_does_what_the_handle_calls_do():
    reqs = _requests(5, seed=22)
    srv = lbm.Server(hbm_budget=64 * GiB, max_sessions=8, quantum=16, variant=0)
    res = _run(srv, reqs)
    srv.close()
    for r, m in zip(reqs, res):
        d, st = _by_hand(r)
        assert m.status == lbm.LBM_OK
        assert m.digest == d
        for f in ("dp", "theta", "dg", "mass"):
            x, y = getattr(m.stats, f), getattr(st, f)
            assert x == y or (np.isnan(x) and np.isnan(y)), f


def test_admission_by_footprint():
    reqs = _requests(8, seed=23)
    sizes = [lbm.lbm_footprint_bytes(r.geom) for r in reqs]
    budget = max(sizes) + min(sizes)
    srv = lbm.Server(hbm_budget=budget, max_sessions=8, quantum=20)
    big = lbm.make_request(2048, 1024, 3, [128, 64, 32, 16], 0.7, 0.03, lbm.LBM_F32,
                           solve_steps=10)
    res = _run(srv, reqs + [big])
    st = srv.stats()
    srv.close()
    assert res[-1].status == lbm.LBM_ENOMEM and res[-1].steps == 0
    assert all(x.status == lbm.LBM_OK for x in res[:-1])
    assert 0 < st.peak_bytes <= budget
    assert st.rejected == 1 and st.completed == len(reqs) + 1
    # the same requests on an unconstrained server give the same bits
    srv = lbm.Server(hbm_budget=64 * GiB, max_sessions=8, quantum=20)
    free = _run(srv, reqs)
    srv.close()
    for a, b in zip(res[:-1], free):
        _same(a, b)


@pytest.mark.parametrize("prec", [lbm.LBM_F64, lbm.LBM_F32, lbm.LBM_F32_S_F16])
def test_footprint_covers_what_a_session_allocates(prec):
    """What a served session does (create, solve, exchange steps, outlet
    statistics) allocates no more than lbm_footprint_bytes, and not much
    less: admission by footprint neither overcommits the device nor wastes
    it."""
    wl = I.HEADLINE_1024x512
    g = lbm.Lattice(wl.types(), wl.tau, wl.u_peak, precision=prec)
    fp = lbm.lbm_footprint_bytes(g.desc)
    created = g.device_bytes()
    assert 0 < created <= fp
    g.run(300, 0.0, 100)
    for seed in (1, 2):
        g.shape_update(frac=0.01, seed=seed)
        g.run(100, 0.0, 100)
    g.stats()
    used = g.device_bytes()
    print(f"prec {prec}: footprint {fp} created {created} after the loop {used}", flush=True)
    assert created <= used <= fp
    assert used >= 0.9 * fp
    g.close()


def test_invalid_requests_are_refused():
    srv = lbm.Server(hbm_budget=GiB, max_sessions=2, quantum=10)
    bad = lbm.make_request(256, 128, 2, [16, 8, 4], 0.7, 0.03, lbm.LBM_F32, solve_steps=10)
    bad.kind = 7
    with pytest.raises(lbm.LbmError):
        srv.submit(bad)
    bad = lbm.make_request(256, 128, 2, [16, 8, 4], 0.7, 0.03, lbm.LBM_F32, solve_steps=-1)
    with pytest.raises(lbm.LbmError):
        srv.submit(bad)
    bad = lbm.make_request(256, 128, 2, [16, 8, 4], 0.4, 0.03, lbm.LBM_F32, solve_steps=10)
    with pytest.raises(lbm.LbmError):
        srv.submit(bad)
    ok = lbm.make_request(256, 128, 2, [16, 8, 4], 0.7, 0.03, lbm.LBM_F32, solve_steps=0)
    (r,) = _run(srv, [ok])
    assert r.status == lbm.LBM_OK and r.steps == 0
    srv.close()
    with pytest.raises(lbm.LbmError):
        lbm.Server(hbm_budget=0)


def test_recycled_memory_does_not_leak_into_results():
    """Destroyed handles hand their blocks to an allocation cache; a new
    lattice of the same size takes them with the previous lattice's data
    still in them.  Its result must not depend on that: the same request
    before and after another lattice of that size has run and been
    destroyed gives the same digest and statistics, bit for bit."""
    c = I.batch_candidates(count=3, seed=33)[0]

    def solve(u_peak, prec, shape=True):
        lat = lbm.Lattice(I.distributor(c.nx, c.ny, c.levels, c.widths), c.tau, u_peak,
                          precision=prec)
        lat.run(150, 0.0, 50)
        if shape:
            lat.shape_update(frac=0.01, seed=3)
            lat.run(40, 0.0, 40)
        flow, st = lat.stats()
        d = lat.digest()
        lat.close()
        # compared as bytes, so that NaN statistics compare equal to themselves
        return np.asarray(flow).tobytes(), np.array([st.dp, st.theta, st.dg]).tobytes(), d

    for prec in (lbm.LBM_F64, lbm.LBM_F32, lbm.LBM_F32_S_F16):
        first = solve(c.u_peak, prec)
        solve(2.0 * c.u_peak, prec)  # different data left in the cached blocks
        again = solve(c.u_peak, prec)
        assert first == again
