"""Pins of the FP64 oracle against facts the paper and the mathematics fix
(closed forms, invariants, special cases, brute force).  CPU only."""
import numpy as np
import pytest

import oracle
from paper_1005_5384_amd import workloads as W


# ---------------------------------------------------------------- direct sum
def test_two_body_closed_form():
    pos = np.array([[0.1, -0.2, 0.3], [0.6, 0.4, -0.2]], np.float32)
    m = np.array([0.25, 0.75], np.float32)
    eps = np.float32(0.05)
    acc, pot = oracle.direct(pos, m, eps)
    d = pos[1].astype(np.float64) - pos[0]
    r2 = d @ d + float(eps) ** 2
    np.testing.assert_allclose(acc[0], float(m[1]) * d / r2 ** 1.5, rtol=1e-14)
    np.testing.assert_allclose(acc[1], -float(m[0]) * d / r2 ** 1.5, rtol=1e-14)
    np.testing.assert_allclose(pot, [-float(m[1]) / r2 ** 0.5, -float(m[0]) / r2 ** 0.5], rtol=1e-14)


def test_cube_corners_point_to_centre():
    # Eight equal masses on the corners of [-1,1]^3: every acceleration points
    # at the centre along the body diagonal, with the closed-form magnitude
    # from 3 edge, 3 face-diagonal and 1 body-diagonal neighbours.
    c = np.array([[x, y, z] for z in (-1, 1) for y in (-1, 1) for x in (-1, 1)], np.float32)
    m = np.full(8, 0.125, np.float32)
    eps = 0.1
    acc, pot = oracle.direct(c, m, eps)
    e2 = np.float64(np.float32(eps)) ** 2
    ax = 0.125 * (2 / (4 + e2) ** 1.5 + 2 * 2 / (8 + e2) ** 1.5 + 2 / (12 + e2) ** 1.5)
    ph = -0.125 * (3 / (4 + e2) ** 0.5 + 3 / (8 + e2) ** 0.5 + 1 / (12 + e2) ** 0.5)
    np.testing.assert_allclose(acc, -np.sign(c) * ax, rtol=1e-13)
    np.testing.assert_allclose(pot, ph, rtol=1e-13)


def test_direct_momentum_conserved():
    pos, m = W.plummer(2048, 7)
    acc, _ = oracle.direct(pos, m, 0.01)
    P = (m[:, None].astype(np.float64) * acc).sum(0)
    scale = (m.astype(np.float64) * np.linalg.norm(acc, axis=1)).sum()
    assert np.all(np.abs(P) <= 1e-12 * scale)


def test_direct_targets_subset_matches_all():
    pos, m = W.plummer(1000, 3)
    a_all, p_all = oracle.direct(pos, m, 0.02)
    tg = np.array([0, 17, 999, 500])
    a, p = oracle.direct(pos, m, 0.02, targets=tg)
    np.testing.assert_array_equal(a, a_all[tg])
    np.testing.assert_array_equal(p, p_all[tg])


def test_direct_plummer_analytic():
    # Truncated Plummer sphere (M = 1, a = 1, cut at Rc = 22.8, renormalised):
    # |a(r)| = r / (f_c (r^2+1)^{3/2}), f_c = Rc^3/(Rc^2+1)^{3/2}, and
    # phi(r) = -1/Rc - [(r^2+1)^{-1/2} - (Rc^2+1)^{-1/2}] / f_c.  Statistical
    # pin: radial-bin means of one realisation within a few percent.
    pos, m = W.plummer(16384, 101)
    acc, pot = oracle.direct(pos, m, 0.01)
    x = pos.astype(np.float64)
    r = np.linalg.norm(x, axis=1)
    ar = -(acc * x).sum(1) / r
    Rc = W.PLUMMER_RCUT
    fc = Rc ** 3 / (Rc ** 2 + 1) ** 1.5
    an = r / (fc * (r * r + 1) ** 1.5)
    edges = np.quantile(r, np.linspace(0.02, 0.95, 12))
    for lo, hi in zip(edges[:-1], edges[1:]):
        s = (r >= lo) & (r < hi)
        assert abs((ar[s] / an[s]).mean() - 1) < 0.05, (lo, hi)
    ph = -1 / Rc - ((r * r + 1) ** -0.5 - (Rc * Rc + 1) ** -0.5) / fc
    assert abs(np.mean(pot / ph) - 1) < 0.01


# ---------------------------------------------------------------- tree
def _invariants(T, pos, m, n_leaf, n_group):
    e = T.export()
    topo, depth, box, mp = e["topo"], e["depth"], e["box"], e["mp"]
    cubes = T.cubes()
    order = e["order"]
    n = pos.shape[0]
    assert np.array_equal(np.sort(order), np.arange(n))
    x = pos.astype(np.float64)[order]
    leaf = topo[:, 1] == 0
    # leaves partition the particles
    cover = np.zeros(n, np.int64)
    for c in np.nonzero(leaf)[0]:
        cover[topo[c, 2]:topo[c, 2] + topo[c, 3]] += 1
    assert np.all(cover == 1)
    assert np.all((topo[leaf, 3] <= n_leaf) | (depth[leaf] == 21))
    assert np.all(topo[~leaf, 3] > n_leaf)
    for c in np.nonzero(~leaf)[0]:
        fc, nc, f, k = topo[c]
        kids = np.arange(fc, fc + nc)
        assert np.all(depth[kids] == depth[c] + 1)
        assert topo[kids[0], 2] == f and topo[kids, 3].sum() == k
        assert np.all(topo[kids[1:], 2] == topo[kids[:-1], 2] + topo[kids[:-1], 3])
        assert abs(mp[kids, 0].sum() - mp[c, 0]) <= 1e-12 * mp[c, 0]
    assert abs(mp[0, 0] - m.astype(np.float64).sum()) <= 1e-12
    # breadth-first numbering: depth is non-decreasing with the cell id
    assert np.all(np.diff(depth) >= 0)
    # particles inside their cell's cube and tight box; box inside the cube
    for c in range(T.n_cells):
        f, k = topo[c, 2], topo[c, 3]
        xs = x[f:f + k]
        lo, s = cubes[c, :3], cubes[c, 3]
        assert np.all(xs >= lo) and np.all(xs < lo + s)
        assert np.array_equal(xs.min(0), box[c, :3]) and np.array_equal(xs.max(0), box[c, 3:])
    # groups: maximal cells with n <= n_group (or leaves), ascending first particle
    g = e["groups"]
    assert np.all((topo[g, 3] <= n_group) | (topo[g, 1] == 0))
    assert np.all(np.diff(topo[g, 2]) > 0)
    assert topo[g, 3].sum() == n


@pytest.mark.parametrize("n,n_leaf,n_group", [(1, 16, 64), (7, 16, 64), (3000, 16, 64),
                                              (3000, 1, 1), (2500, 8, 32)])
def test_tree_invariants(n, n_leaf, n_group):
    pos, m = W.plummer(n, 11 + n)
    T = oracle.Tree(pos, m, n_leaf, n_group)
    _invariants(T, pos, m, n_leaf, n_group)


def test_tree_coincident_particles_stop_at_depth_21():
    pos = np.zeros((40, 3), np.float32)
    pos[20:] = [1.0, 2.0, -1.0]
    m = np.full(40, 0.025, np.float32)
    T = oracle.Tree(pos, m, 4, 8)
    e = T.export()
    assert T.max_depth == 21
    leaf = e["topo"][:, 1] == 0
    assert sorted(e["topo"][leaf, 3].tolist()) == [20, 20]
    # each stack of coincident particles is one group (a depth-21 leaf)
    assert sorted(e["topo"][e["groups"], 3].tolist()) == [20, 20]
    _invariants(T, pos, m, 4, 8)


def test_tree_plane_tie_goes_upper():
    # Extent 4 gives a root cube of side 8 centred on the box centre 2, i.e.
    # [-2, 6)^3 with its midplanes at 2: the particle exactly on them goes to
    # the upper octant, together with [4,4,4].
    pos = np.array([[0, 0, 0], [4, 4, 4], [2, 2, 2], [1, 1, 1]], np.float32)
    m = np.full(4, 0.25, np.float32)
    T = oracle.Tree(pos, m, 1, 1)
    e = T.export()
    assert e["cube"][3] == 8.0 and np.all(e["cube"][:3] == -2.0)
    top = e["topo"][0]
    kids = np.arange(top[0], top[0] + top[1])
    members = [set(e["order"][e["topo"][k, 2]:e["topo"][k, 2] + e["topo"][k, 3]].tolist())
               for k in kids]
    assert members == [{0, 3}, {1, 2}]
    assert np.all(T.cubes()[kids[1], :3] == 2.0)


def test_moments_closed_forms():
    # dumbbell of masses m at +-d x: Q = m d^2 diag(4, -2, -2), com = 0
    d, mm = 0.75, 0.5
    pos = np.array([[d, 0, 0], [-d, 0, 0]], np.float32)
    T = oracle.Tree(pos, np.full(2, mm, np.float32), 64, 64)
    mp = T.export()["mp"][0]
    np.testing.assert_allclose(mp[:4], [2 * mm, 0, 0, 0], atol=1e-15)
    np.testing.assert_allclose(mp[4:], mm * d * d * np.array([4, -2, -2, 0, 0, 0]), atol=1e-15)
    # eight cube corners: Q = 0
    c = np.array([[x, y, z] for z in (-1, 1) for y in (-1, 1) for x in (-1, 1)], np.float32) + 3
    T = oracle.Tree(c, np.full(8, 0.125, np.float32), 64, 64)
    mp = T.export()["mp"][0]
    np.testing.assert_allclose(mp[1:4], [3, 3, 3], rtol=1e-15)
    np.testing.assert_allclose(mp[4:], 0, atol=1e-14)
    # single particle: com = x exactly, Q = 0
    p = np.array([[0.3, -1.7, 2.2]], np.float32)
    T = oracle.Tree(p, np.ones(1, np.float32), 16, 64)
    mp = T.export()["mp"][0]
    assert np.array_equal(mp[1:4], p[0].astype(np.float64)) and np.all(mp[4:] == 0)


def test_quadrupole_convergence_slope():
    # The particle-cell expansion's relative error falls with slope ~ -3 in
    # log(l/d) with the quadrupole and ~ -2 with the monopole alone; a wrong
    # sign or factor in the quadrupole terms leaves slope -2.
    rng = np.random.default_rng(5)
    src = (rng.uniform(-0.5, 0.5, (200, 3)) * [1.0, 0.6, 0.3]).astype(np.float32)
    ms = rng.uniform(0.5, 1.5, 200).astype(np.float32)
    dirn = np.array([0.48, 0.6, 0.64])
    ds = np.array([4.0, 8.0, 16.0, 32.0])
    errs = {True: [], False: []}
    perrs = {True: [], False: []}
    for dd in ds:
        tgt = dirn * dd
        ex_a = np.zeros(3)
        ex_p = 0.0
        for j in range(200):
            R = src[j].astype(np.float64) - tgt
            r = np.sqrt(R @ R)
            ex_a += ms[j] * R / r ** 3
            ex_p -= ms[j] / r
        for q in (True, False):
            a, p = oracle.multipole_eval(src, ms, tgt, 1e-12, use_quad=q)
            errs[q].append(np.linalg.norm(a - ex_a) / np.linalg.norm(ex_a))
            perrs[q].append(abs(p - ex_p) / abs(ex_p))
    sq = np.polyfit(np.log(ds), np.log(errs[True]), 1)[0]
    sm = np.polyfit(np.log(ds), np.log(errs[False]), 1)[0]
    assert -3.4 < sq < -2.6, sq
    assert -2.4 < sm < -1.6, sm
    # the same law for the potential: -M/r - s/(2 r^5) leaves an octupole
    # error; a wrong sign or factor of the s term leaves the quadrupole's
    psq = np.polyfit(np.log(ds), np.log(perrs[True]), 1)[0]
    psm = np.polyfit(np.log(ds), np.log(perrs[False]), 1)[0]
    assert -3.4 < psq < -2.6, psq
    assert -2.4 < psm < -1.6, psm


def _dumbbell_field(half, m, direction, d):
    """Monopole + quadrupole field of two masses m at +-half (a 3-vector) seen
    at distance d along `direction`: the oracle's particle-cell evaluation."""
    pos = np.array([half, -np.asarray(half)], np.float32)
    u = np.asarray(direction, np.float64)
    return oracle.multipole_eval(pos, np.full(2, m, np.float32), u / np.linalg.norm(u) * d, 1e-12)


@pytest.mark.parametrize("d", [3.0, 5.0, 12.0])
def test_dumbbell_multipole_closed_form(d):
    # Two masses m at +-b from their centre.  The exact potential on the axis
    # is -m/(d-b) - m/(d+b) = -(2m/d)(1 + b^2/d^2 + b^4/d^4 + ...), off the axis
    # (perpendicular) -2m/sqrt(d^2+b^2) = -(2m/d)(1 - b^2/(2 d^2) + ...); the
    # monopole + quadrupole expansion keeps the first two terms of each, and
    # the accelerations are the radial derivatives of the same series:
    #   on the axis:    phi = -2m/d - 2 m b^2/d^3,  a_r = -2m/d^2 - 6 m b^2/d^4
    #   perpendicular:  phi = -2m/d + m b^2/d^3,    a_r = -2m/d^2 + 3 m b^2/d^4
    # (a_r: the component along the direction from the centre to the target).
    m = 0.75
    for half, b2 in (([0.5, 0.0, 0.0], 0.25),           # along x: Q diagonal
                     ([0.5, 0.5, 0.0], 0.5),            # diagonal: Q_xy != 0
                     ([0.25, -0.5, 0.5], 0.5625)):      # general: every Q component
        h = np.asarray(half, np.float64)
        perp = np.cross(h, [0.3, 0.7, 0.1])
        for direction, phi_ref, ar_ref in (
                (h, -2 * m / d - 2 * m * b2 / d ** 3, -2 * m / d ** 2 - 6 * m * b2 / d ** 4),
                (perp, -2 * m / d + m * b2 / d ** 3, -2 * m / d ** 2 + 3 * m * b2 / d ** 4)):
            a, phi = _dumbbell_field(half, m, direction, d)
            u = direction / np.linalg.norm(direction)
            np.testing.assert_allclose(phi, phi_ref, rtol=1e-12)
            np.testing.assert_allclose(a @ u, ar_ref, rtol=1e-12)
            # no tangential component on these two symmetry lines
            assert np.linalg.norm(a - (a @ u) * u) <= 1e-12 * abs(ar_ref)


def test_single_particle_cell_equals_pair():
    p = np.array([[0.2, 0.1, -0.3]], np.float32)
    a, ph = oracle.multipole_eval(p, np.array([0.7], np.float32), [1.0, 2.0, 0.5], 0.05)
    R = p[0].astype(np.float64) - [1.0, 2.0, 0.5]
    r2 = R @ R + np.float64(np.float32(0.05)) ** 2
    np.testing.assert_allclose(a, 0.7 * R / r2 ** 1.5 * np.float32(0.7) / 0.7, rtol=1e-7)
    np.testing.assert_allclose(ph, -np.float64(np.float32(0.7)) / r2 ** 0.5, rtol=1e-14)


# ---------------------------------------------------------------- opening test
def test_mac_adversarial():
    gmin = np.array([0, 0, 0], np.float32)
    gmax = np.array([1, 1, 1], np.float32)
    # d = 2 exactly from the box (boundary centre at x = 3), theta = 0.5: d*theta == l
    # at l = 1 is a tie and is accepted (strict test); a hair larger l opens.
    assert not oracle.mac_open(gmin, gmax, [3, 0.5, 0.5, 1.0], 0.5)
    assert oracle.mac_open(gmin, gmax, [3, 0.5, 0.5, np.nextafter(np.float32(1), np.float32(2))], 0.5)
    # centre inside the group box: d2 == 0 opens, even for l = 0
    assert oracle.mac_open(gmin, gmax, [0.5, 0.5, 0.5, 0.0], 0.5)
    assert oracle.mac_open(gmin, gmax, [1.0, 1.0, 1.0, 0.0], 0.0)
    # l = 0 outside the box: accepted at every theta
    assert not oracle.mac_open(gmin, gmax, [1.5, 0.5, 0.5, 0.0], 1.0)
    # denormal distance: t^2 underflows to 0 -> d2 == 0 -> open
    z = np.zeros(3, np.float32)
    assert oracle.mac_open(z, z, [np.float32(1e-40), 0, 0, 1e-30], 0.5)
    # l^2 underflows to 0 while d2 does not: accepted
    assert not oracle.mac_open(z, z, [np.float32(1e-10), 0, 0, 1e-30], 0.5)
    # theta = 0: every l > 0 cell is opened however far it is (distances stay
    # far below FP32 overflow; the library rejects coordinates >= 2^60)
    assert oracle.mac_open(gmin, gmax, [1e15, 0, 0, 1e-3], 0.0)


def test_mac_group_overlap_always_opens():
    # A cell whose boundary cube meets the group box is opened for theta <= 1.
    rng = np.random.default_rng(2)
    for _ in range(2000):
        gmin = rng.uniform(-1, 0, 3).astype(np.float32)
        gmax = (gmin + rng.uniform(0, 1, 3)).astype(np.float32)
        l = np.float32(rng.uniform(0.01, 2))
        p = rng.uniform(gmin, gmax)  # a point of the box inside the cube
        cb = (p + rng.uniform(-0.5, 0.5, 3) * l).astype(np.float32)
        assert oracle.mac_open(gmin, gmax, [*cb, l], 1.0)


# ---------------------------------------------------------------- lists
@pytest.mark.parametrize("theta", [0.0, 0.2, 0.5, 0.75, 1.0])
def test_lists_walk_equals_characterisation(theta):
    pos, m = W.plummer(600, 21)
    T = oracle.Tree(pos, m, 4, 16)
    a = T.lists(theta)
    b = T.lists_brute(theta)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


def test_lists_cover_every_particle_once():
    # For each group, the accepted cells and opened leaves together hold every
    # particle exactly once, and the group's own leaves are in its leaf list.
    pos, m = W.plummer(3000, 5)
    T = oracle.Tree(pos, m, 8, 32)
    e = T.export()
    topo = e["topo"]
    c_off, c_ids, l_off, l_ids = T.lists(0.6)
    for g in range(T.n_groups):
        cover = np.zeros(pos.shape[0], np.int64)
        for c in np.concatenate([c_ids[c_off[g]:c_off[g + 1]], l_ids[l_off[g]:l_off[g + 1]]]):
            cover[topo[c, 2]:topo[c, 2] + topo[c, 3]] += 1
        assert np.all(cover == 1)
        gc = e["groups"][g]
        f, k = topo[gc, 2], topo[gc, 3]
        assert np.all(cover[f:f + k] == 1)
        own = set(range(f, f + k))
        for c in c_ids[c_off[g]:c_off[g + 1]]:
            assert not own & set(range(topo[c, 2], topo[c, 2] + topo[c, 3]))


def test_lists_root_leaf():
    pos, m = W.plummer(10, 1)
    T = oracle.Tree(pos, m, 16, 64)
    c_off, c_ids, l_off, l_ids = T.lists(0.5)
    assert T.n_cells == 1 and c_ids.size == 0 and list(l_ids) == [0]


# ---------------------------------------------------------------- tree forces
def test_theta_zero_equals_direct():
    pos, m = W.plummer(2048, 9)
    T = oracle.Tree(pos, m, 8, 32)
    a, p = T.forces(0.0, 0.01)
    ad, pd = oracle.direct(pos, m, 0.01)
    assert np.max(oracle.rel_err(a, ad)) < 1e-12
    assert np.max(oracle.rel_err(p, pd)) < 1e-12


def test_coincident_cells_theta_zero_equals_direct():
    # l = 0 cells (coincident particles) go through the p-c path as exact point masses.
    rng = np.random.default_rng(4)
    base = rng.normal(size=(50, 3)).astype(np.float32)
    pos = np.repeat(base, 3, axis=0)
    m = rng.uniform(0.5, 1, 150).astype(np.float32)
    T = oracle.Tree(pos, m, 2, 4)
    a, p = T.forces(0.0, 0.01)
    ad, pd = oracle.direct(pos, m, 0.01)
    assert np.max(oracle.rel_err(a, ad)) < 1e-12
    assert np.max(oracle.rel_err(p, pd)) < 1e-12


def test_error_grows_like_theta4():
    # Sec. 3.1: the median relative error grows roughly like theta^4.
    pos, m = W.plummer(16384, 101)
    T = oracle.Tree(pos, m, 16, 64)
    ad, _ = oracle.direct(pos, m, 0.01)
    th = np.array([0.3, 0.5, 0.75])
    med = [np.median(oracle.rel_err(T.forces(t, 0.01)[0], ad)) for t in th]
    slope = np.polyfit(np.log(th), np.log(med), 1)[0]
    assert 3.0 < slope < 5.0, slope


def test_forces_subset_matches_full():
    pos, m = W.plummer(4000, 8)
    T = oracle.Tree(pos, m, 16, 64)
    a, p = T.forces(0.5, 0.01)
    sel = np.array([0, 3, T.n_groups - 1])
    a2, p2 = T.forces(0.5, 0.01, groups=sel)
    ok = ~np.isnan(p2)
    assert ok.sum() > 0
    assert np.array_equal(a2[ok], a[ok]) and np.array_equal(p2[ok], p[ok])


# ---------------------------------------------------------------- statistics
def test_percentile_nearest_rank():
    x = np.arange(1, 101, dtype=float)[::-1]
    assert oracle.percentile_nr(x, 0.5) == 50
    assert oracle.percentile_nr(x, 0.99) == 99
    assert oracle.percentile_nr(x, 1.0) == 100
    assert oracle.percentile_nr([3.0], 0.99) == 3.0
    assert oracle.percentile_nr([1.0, 2.0, 3.0], 0.5) == 2.0


def test_diagnostics_direct():
    pos, m = W.plummer(1024, 12)
    a, p = oracle.direct(pos, m, 0.01)
    P, Wp = oracle.diagnostics(m, a, p)
    assert np.all(np.abs(P) < 1e-14)
    assert np.isclose(Wp, 0.5 * np.sum(m.astype(np.float64) * p), rtol=1e-14)
    # Untruncated, unsoftened Plummer: W = -3 pi / 32; N = 1024 is near it.
    assert abs(Wp / (-3 * np.pi / 32) - 1) < 0.05


def test_forces_from_given_lists_equal_own_walk():
    pos, m = W.plummer(2048, 77)
    T = oracle.Tree(pos, m, 8, 32)
    a, p = T.forces(0.6, 0.01)
    b, q = T.forces_lists(T.lists(0.6), 0.01)
    assert np.array_equal(a, b) and np.array_equal(p, q)
    # lists of another angle give that angle's forces
    c, _ = T.forces_lists(T.lists(0.4), 0.01)
    d, _ = T.forces(0.4, 0.01)
    assert np.array_equal(c, d)


def test_lists_of_selected_groups_equal_full_lists():
    # the group-selected walk (used where full lists would not fit in host
    # memory) gives exactly the full walk's lists of those groups, in the
    # order asked for, also under the learned criterion; bad indices rejected
    pos, m = W.plummer(20000, 5)
    O = oracle.Tree(pos, m, 16, 64)
    sel = np.array([3, 0, 17, O.n_groups - 1, 3], np.int32)
    for theta in (0.3, 0.6):
        full = O.lists(theta)
        part = O.lists(theta, groups=sel)
        for j, g in enumerate(sel):
            for k in (0, 2):
                a = full[k + 1][full[k][g]:full[k][g + 1]]
                b = part[k + 1][part[k][j]:part[k][j + 1]]
                assert np.array_equal(a, b)
    P = np.random.default_rng(0).normal(0, 0.1, 5057)
    lf, fb = O.lists_learned(0.6, 0.4, 0.8, -3.0, 1.0, params=P)
    lp, fbp = O.lists_learned(0.6, 0.4, 0.8, -3.0, 1.0, params=P, groups=sel)
    for j, g in enumerate(sel):
        for k in (0, 2):
            assert np.array_equal(lf[k + 1][lf[k][g]:lf[k][g + 1]], lp[k + 1][lp[k][j]:lp[k][j + 1]])
        assert fb[g] == fbp[j]
    with pytest.raises(ValueError):
        O.lists(0.5, groups=np.array([O.n_groups], np.int32))
    with pytest.raises(ValueError):
        O.lists_learned(0.6, 0.4, 0.8, -3.0, 1.0, params=P, groups=np.array([-1], np.int32))
