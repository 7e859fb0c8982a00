"""Synthetic workload generator: structure of the distributor (Sec. 3.2) and
the channel-width scaling law (Eq. 8) against Table 1."""
import os
from collections import deque

import numpy as np
import pytest

from paper_1303_0107_amd import inputs as I

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _runs(col, value):
    runs, y = [], 0
    while y < len(col):
        if col[y] == value:
            y0 = y
            while y < len(col) and col[y] == value:
                y += 1
            runs.append((y0, y - 1))
        else:
            y += 1
    return runs


def _reachable(t, start):
    ny, nx = t.shape
    seen = np.zeros_like(t, bool)
    q = deque([start])
    seen[start] = True
    while q:
        y, x = q.popleft()
        for dy, dx in ((1, 0), (-1, 0), (0, 1), (0, -1)):
            a, b = y + dy, x + dx
            if 0 <= a < ny and 0 <= b < nx and not seen[a, b] and t[a, b] != 0:
                seen[a, b] = True
                q.append((a, b))
    return seen


@pytest.mark.parametrize("w", [I.CORRECTNESS_128x64, I.HEADLINE_1024x512, I.PRECISION_2048x1024])
def test_distributor_structure(w):
    t = w.types()
    assert t.shape == (w.ny, w.nx)
    assert not t[0].any() and not t[-1].any()
    inl = _runs(t[:, 0], I.INLET)
    out = _runs(t[:, -1], I.OUTLET)
    assert len(inl) == 1 and inl[0][1] - inl[0][0] + 1 == w.widths[0]
    assert len(out) == 2 ** w.levels
    assert all(b - a + 1 == w.widths[-1] for a, b in out)
    # equally spaced outlets (Sec. 3.2)
    starts = np.diff([a for a, _ in out])
    assert len(set(starts.tolist())) == 1
    assert np.array_equal(t, t[::-1])  # mirror symmetric about mid-height
    seen = _reachable(t, (inl[0][0], 0))
    assert all(seen[a, w.nx - 1] for a, _ in out)
    assert seen[t != 0].all()  # no disconnected fluid
    assert set(np.unique(t[:, 1:-1]).tolist()) <= {0, 1}


def test_channel_and_box():
    t = I.channel(16, 8)
    assert (t[1:-1, 0] == 2).all() and (t[1:-1, -1] == 3).all()
    assert (t[1:-1, 1:-1] == 1).all() and not t[0].any() and not t[-1].any()
    b = I.closed_box(10, 6)
    assert not b[0].any() and not b[:, 0].any() and (b[1:-1, 1:-1] == 1).all()


def test_width_law_reproduces_table1():
    """Eq. 8 with h = 10 mm from w4 = 2 mm gives Table 1's widths within 1%
    (the table lists them in reverse order against the generation index)."""
    rows = [l.split() for l in open(os.path.join(GOLDEN, "table1_channel_widths.txt"))
            if l.strip() and not l.startswith("#")]
    table = {int(r[0]): float(r[1]) for r in rows}
    ws = I.width_law_chain(10.0, table[4], 3)  # w1..w4
    for k in (1, 2, 3, 4):
        assert ws[k - 1] == pytest.approx(table[k], rel=0.01)
    # chaining from the rounded table values lands closer still
    assert I.width_law_ratio(10.0, table[3]) == pytest.approx(table[2], rel=0.005)
    assert I.width_law_ratio(10.0, table[2]) == pytest.approx(table[1], rel=0.005)


def test_width_law_deep_channel_limit():
    """For h >> w Eq. 8 tends to Murray's 2D law w_{k+1}/w_k = 2^(-1/2)."""
    assert I.width_law_ratio(1e9, 1.0) == pytest.approx(2 ** 0.5, rel=1e-6)


def test_invalid_widths():
    with pytest.raises(ValueError):
        I.distributor(128, 64, 3, [8, 8, 8, 7])  # 64/8 < 7 + 2
    with pytest.raises(ValueError):
        I.distributor(128, 64, 2, [8, 1, 4])


def test_batch_candidates_reproducible_and_valid():
    a = I.batch_candidates(32, seed=4)
    b = I.batch_candidates(32, seed=4)
    assert [(c.nx, c.ny, c.levels, c.widths, c.tau) for c in a] == \
        [(c.nx, c.ny, c.levels, c.widths, c.tau) for c in b]
    for c in a:
        assert 128 <= c.nx <= 1024 and 64 <= c.ny <= 512 and c.nx % 64 == 0
        assert 2 <= c.levels <= 4 and 0.55 <= c.tau <= 1.0
        t = c.types()
        assert len(_runs(t[:, -1], I.OUTLET)) == 2 ** c.levels


def test_serving_requests_follow_their_recipe():
    reqs = I.serving_requests(rate=50.0, seconds=20.0, seed=5)
    again = I.serving_requests(rate=50.0, seconds=20.0, seed=5)
    assert [(r.t, r.workload.nx, r.kind) for r in reqs] == [(r.t, r.workload.nx, r.kind) for r in again]
    assert 800 < len(reqs) < 1200                      # Poisson, mean 1000
    t = np.array([r.t for r in reqs])
    assert np.all(np.diff(t) > 0) and t[-1] < 20.0
    for r in reqs:
        w = r.workload
        assert w.nx % 64 == 0 and 256 <= w.nx <= 4096 and w.ny == w.nx // 2
        assert 2 <= w.levels <= 4 and len(w.widths) == w.levels + 1
        assert 0.55 <= w.tau <= 1.0 and 0.02 <= w.u_peak <= 0.06
        assert r.storage in ("f32", "f16") and r.kind in ("solve", "optimize")
        steps = r.solve_steps + r.iterations * r.steps_per_iteration
        assert steps == (500 if r.kind == "solve" else 900)
    f32 = np.mean([r.storage == "f32" for r in reqs])
    solve = np.mean([r.kind == "solve" for r in reqs])
    assert 0.4 < f32 < 0.6 and 0.4 < solve < 0.6
