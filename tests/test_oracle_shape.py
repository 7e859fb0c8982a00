"""Pins of the oracle's exchange step (Sec. 2.2, Eqs. 5-6; Sec. 2.3 step 3).

Hand-built cases whose answer follows from the criteria by inspection, the
invariants the step must keep (constant fluid volume, |R| = |A|), and a
brute-force rank count (an O(n^2) algorithm unlike the oracle's sort) for the
selection and its tie-breaking.
"""
import math

import numpy as np
import pytest

from paper_1303_0107_amd import inputs as I

E4 = [(1, 0), (0, 1), (-1, 0), (0, -1)]


def _channel_field(nx=12, ny=10, rows=(3, 6)):
    """Horizontal channel on rows[0]..rows[1], solid elsewhere; no ports."""
    t = np.zeros((ny, nx), np.uint8)
    t[rows[0]:rows[1] + 1, :] = 1
    t[:, 0] = np.where(t[:, 0] != 0, 2, 0)
    t[:, -1] = np.where(t[:, -1] != 0, 3, 0)
    rho = np.where(t != 0, 1.0, 0.0)
    ux = np.where(t != 0, 0.02, 0.0)
    uy = np.zeros_like(ux)
    return t, rho, ux, uy


def test_dead_end_pocket_is_filled_first(orc):
    """Fluid cells of a stagnant side pocket (u = 0, lowest dynamic pressure
    q = rho |u|^2 / 2, Eq. 6) are the first to become solid."""
    t, rho, ux, uy = _channel_field()
    t[7:9, 5] = 1  # a 2-cell pocket above the channel at x = 5
    ux[7:9, 5] = 0.0
    nf = int((t == 1).sum())
    frac = 2.0 / nf  # K = 2
    new, r = orc.shape_select(t, rho, ux, uy, frac=frac, seed=1)
    assert r.k_eff == 2
    got = {(int(i) % t.shape[1], int(i) // t.shape[1]) for i in r.removed}
    assert got == {(5, 7), (5, 8)}
    assert new[7, 5] == 0 and new[8, 5] == 0


def test_wall_beside_fastest_tangential_flow_is_eroded_first(orc):
    """A solid cell whose fluid neighbour across a horizontal face moves
    fastest along that face suffers the largest viscous stress (Eq. 5) and is
    the first to become fluid."""
    t, rho, ux, uy = _channel_field()
    ux[6, 7] = 0.1  # top fluid row, below the solid cell (7, 7)
    nf = int((t == 1).sum())
    new, r = orc.shape_select(t, rho, ux, uy, frac=1.0 / nf, seed=3)
    assert r.k_eff == 1
    assert int(r.added[0]) == 7 * t.shape[1] + 7
    assert new[7, 7] == 1


def test_stress_uses_the_tangential_velocity(orc):
    """Eq. 5 pairs u with the y spacing and v with the x spacing: across a
    vertical face (E/W neighbour) only u_y shears the wall, across a
    horizontal face (N/S neighbour) only u_x.  A solid cell facing a fast
    normal flow therefore has zero stress."""
    t = np.zeros((9, 9), np.uint8)
    t[4, 1:5] = 1           # stub ending at x = 4; solid cell (5, 4) faces its tip
    t[1:4, 4] = 1           # vertical stub below, so (5, 4)'s E/W faces are the only contact
    rho = np.where(t != 0, 1.0, 0.0)
    ux = np.zeros((9, 9))
    uy = np.zeros((9, 9))
    ux[4, 4] = 0.3          # normal to the face between (4, 4) and (5, 4)
    uy[4, 4] = 0.0
    uy[2, 4] = 0.05         # tangential along the faces of (3, 2) and (5, 2)
    _, r = orc.shape_select(t, rho, ux, uy, frac=1.0, seed=0, band_x=1, band_y=1)
    nx = t.shape[1]
    keys = _solid_keys_paper(t, ux, uy)
    # (5, 4) touches (4, 4) on its W face: key = |u_y(4, 4)| = 0
    assert keys[(5, 4)] == 0.0
    # (4, 5) sits above (4, 4): key = |u_x(4, 4)| = 0.3, the largest
    assert keys[(4, 5)] == pytest.approx(0.3)
    assert int(r.added[0]) == 5 * nx + 4


def _solid_keys_paper(t, ux, uy):
    ny, nx = t.shape
    keys = {}
    for y in range(1, ny - 1):
        for x in range(1, nx - 1):
            if t[y, x] != 0:
                continue
            k, touch = 0.0, False
            for dx, dy in E4:
                if t[y + dy, x + dx] != 0:
                    touch = True
                    k += abs(uy[y + dy, x + dx]) if dx else abs(ux[y + dy, x + dx])
            if touch:
                keys[(x, y)] = k
    return keys


def _brute_force(t, rho, ux, uy, frac, seed, bx, by, criterion, orc):
    """Selection by explicit rank counting over the candidate sets."""
    ny, nx = t.shape
    cf, cs = [], []
    for y in range(by, ny - by):
        for x in range(bx, nx - bx):
            n = y * nx + x
            nb = [t[y + dy, x + dx] for dx, dy in E4]
            h = orc.splitmix64(seed + n)
            if t[y, x] == 1 and any(v == 0 for v in nb):
                s = ux[y, x] ** 2 + uy[y, x] ** 2
                cf.append((rho[y, x] * s if criterion == 0 else s, h, n))
            elif t[y, x] == 0 and any(v != 0 for v in nb):
                terms = []
                for dx, dy in E4:
                    if t[y + dy, x + dx] != 0:
                        a, b = ux[y + dy, x + dx], uy[y + dy, x + dx]
                        terms.append((abs(b) if dx else abs(a)) if criterion == 0 else a * a + b * b)
                k = 0.0
                if criterion == 0:
                    for v in terms:
                        k = k + v
                else:
                    k = max(terms)
                cs.append((k, h, n))
    nf = int((t == 1).sum())
    K = max(1, math.floor(frac * nf))
    keff = min(K, len(cf), len(cs))

    def ranks(c, desc):
        out = []
        for a in c:
            r = 0
            for b in c:
                if desc:
                    less = (b[0] > a[0]) or (b[0] == a[0] and (b[1], b[2]) < (a[1], a[2]))
                else:
                    less = (b[0] < a[0]) or (b[0] == a[0] and (b[1], b[2]) < (a[1], a[2]))
                r += less
            out.append(r)
        return out

    rf, rs = ranks(cf, False), ranks(cs, True)
    removed = [None] * keff
    added = [None] * keff
    for c, r in zip(cf, rf):
        if r < keff:
            removed[r] = c[2]
    for c, r in zip(cs, rs):
        if r < keff:
            added[r] = c[2]
    return keff, removed, added


@pytest.mark.parametrize("criterion", [0, 1])
@pytest.mark.parametrize("seed", [1, 7])
def test_selection_matches_brute_force_rank_count(orc, criterion, seed):
    t = I.CORRECTNESS_128x64.types()[:, :64].copy()
    t[:, -1] = np.where(t[:, -1] != 0, 3, 0)
    rho, ux, uy = I.random_field(t, seed)
    # quantise so that exact key ties occur and the hash decides
    ux = np.round(ux, 2)
    uy = np.round(uy, 2)
    new, r = orc.shape_select(t, rho, ux, uy, frac=0.05, seed=seed, criterion=criterion)
    keff, rem, add = _brute_force(t, rho, ux, uy, 0.05, seed, 2, 1, criterion, orc)
    assert r.k_eff == keff
    assert list(r.removed) == rem
    assert list(r.added) == add
    assert r.mass_removed == math.fsum(rho.ravel()[rem]) or \
        abs(r.mass_removed - math.fsum(rho.ravel()[rem])) < 1e-14 * keff


def test_all_equal_keys_fall_back_to_the_hash(orc):
    t = I.CORRECTNESS_128x64.types()
    z = np.zeros(t.shape)
    rho = np.where(t != 0, 1.0, 0.0)
    seed = 12345
    _, r = orc.shape_select(t, rho, z, z, frac=0.01, seed=seed)
    nx = t.shape[1]
    # every interface fluid cell has key 0: the removed ones are those with
    # the smallest hashes
    cand = []
    for y in range(1, t.shape[0] - 1):
        for x in range(2, nx - 2):
            if t[y, x] == 1 and any(t[y + dy, x + dx] == 0 for dx, dy in E4):
                cand.append((orc.splitmix64(seed + y * nx + x), y * nx + x))
    cand.sort()
    assert list(r.removed) == [c[1] for c in cand[:r.k_eff]]


def test_constant_volume_and_counts(orc):
    """Equal numbers of cells change phase (constant void volume, Sec. 2.2):
    K = max(1, floor(frac N_f)), |R| = |A| = K_eff, N_f unchanged, R taken
    from fluid interface cells and A from solid interface cells."""
    t = I.CORRECTNESS_128x64.types()
    rho, ux, uy = I.random_field(t, 3)
    nf = int((t == 1).sum())
    new, r = orc.shape_select(t, rho, ux, uy, frac=0.01, seed=2)
    assert r.k_eff == max(1, math.floor(0.01 * nf)) == 17
    assert r.n_fluid_before == r.n_fluid_after == nf == int((new == 1).sum())
    assert len(set(r.removed)) == len(set(r.added)) == r.k_eff
    flat_old, flat_new = t.ravel(), new.ravel()
    assert all(flat_old[i] == 1 and flat_new[i] == 0 for i in r.removed)
    assert all(flat_old[i] == 0 and flat_new[i] == 1 for i in r.added)
    changed = np.flatnonzero(flat_old != flat_new)
    assert set(changed) == set(r.removed) | set(r.added)
    assert r.mass_added == float(r.k_eff)
    # never inside the frozen band, never a port
    ny, nx = t.shape
    for i in list(r.removed) + list(r.added):
        x, y = i % nx, i // nx
        assert 2 <= x <= nx - 3 and 1 <= y <= ny - 2


def test_warm_and_cold_reinitialisation(orc):
    _, _, _, w = orc.velocity_set()
    t = I.CORRECTNESS_128x64.types()
    lat = orc.Lattice(t, 0.8, 0.05)
    lat.run(500)
    before = lat.fs.copy()
    r = lat.shape_update(frac=0.01, seed=1, reinit=orc.WARM)
    ny, nx = t.shape
    for i in r.added:
        assert np.array_equal(lat.fs[:, i // nx, i % nx], w)
    for i in r.removed:
        assert not lat.fs[:, i // nx, i % nx].any()
    mask = np.ones((ny, nx), bool)
    mask.ravel()[np.concatenate([r.removed, r.added])] = False
    assert np.array_equal(lat.fs[:, mask], before[:, mask])
    lat2 = orc.Lattice(t, 0.8, 0.05)
    lat2.run(500)
    lat2.shape_update(frac=0.01, seed=1, reinit=orc.COLD)
    ns = lat2.types != 0
    assert np.array_equal(lat2.fs[:, ns], np.repeat(w[:, None], ns.sum(), 1))


def test_nan_key_is_an_error(orc):
    t = I.CORRECTNESS_128x64.types()
    rho, ux, uy = I.random_field(t, 3)
    ny, nx = t.shape
    y, x = next((y, x) for y in range(1, ny - 1) for x in range(2, nx - 2)
                if t[y, x] == 1 and t[y + 1, x] == 0)
    ux[y, x] = np.nan
    with pytest.raises(ValueError):
        orc.shape_select(t, rho, ux, uy, frac=0.01, seed=2)
