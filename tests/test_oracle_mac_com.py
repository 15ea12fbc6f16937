"""Pins of the oracle's centre-of-mass offset opening test (open iff
d(com, group box) < l / theta + |com - cb|, in FP32): it reduces to the
boundary-centre test when the centres coincide, closed-form ties on an axis,
the walk equals the walk-free characterisation, every cell holding a group
particle is opened for theta <= 0.57, and at theta = 0 the lists give the
direct sum."""
import numpy as np
import pytest

import oracle
from paper_1005_5384_amd import workloads as W


def _com32(O):
    return O.export()["mp"][:, 1:4].astype(np.float32)


def test_zero_offset_is_the_boundary_test():
    rng = np.random.default_rng(5)
    for _ in range(3000):
        gmin = rng.uniform(-1, 1, 3).astype(np.float32)
        gmax = (gmin + rng.uniform(0, 0.5, 3)).astype(np.float32)
        geo = np.concatenate([rng.uniform(-3, 3, 3), rng.uniform(0, 2, 1)]).astype(np.float32)
        th = float(rng.uniform(0, 0.57))
        assert oracle.mac_open_com(gmin, gmax, geo[:3], geo, th) == oracle.mac_open(gmin, gmax, geo, th)


@pytest.mark.parametrize("com_x,theta,expect", [
    (5.0, 0.5, False),   # d = 5, l' = 2.5: 25 * 0.25 == 6.25, a tie accepts
    (5.0, 0.49, True),   # open iff 5 theta < 2 + theta, i.e. theta < 0.5
    (5.0, 0.51, False),
    (3.0, 0.57, True),   # d = 3: open iff 3 theta < 2 + theta, i.e. theta < 1
    (4.0, 0.5, False),   # no offset: the boundary test's own tie (4 * 0.5 == 2)
    (4.0, 0.49, True),
])
def test_closed_form_on_axis(com_x, theta, expect):
    # group box = the origin; boundary centre (4, 0, 0), side 2; com on the x axis
    z = np.zeros(3, np.float32)
    geo = np.array([4.0, 0.0, 0.0, 2.0], np.float32)
    com = np.array([com_x, 0.0, 0.0], np.float32)
    assert oracle.mac_open_com(z, z, com, geo, theta) == expect


def test_offset_makes_the_test_depend_on_the_side_of_the_offset():
    # an offset toward the group opens at angles where the boundary test accepts
    z = np.zeros(3, np.float32)
    geo = np.array([4.0, 0.0, 0.0, 2.0], np.float32)
    near, far = np.array([3.0, 0, 0], np.float32), np.array([5.0, 0, 0], np.float32)
    for th in (0.52, 0.55, 0.57):
        assert not oracle.mac_open(z, z, geo, th)
        assert oracle.mac_open_com(z, z, near, geo, th)
        assert not oracle.mac_open_com(z, z, far, geo, th)


@pytest.mark.parametrize("n,n_leaf,n_group,seed", [(500, 4, 16, 1), (2500, 8, 64, 2),
                                                   (3000, 1, 1, 3)])
@pytest.mark.parametrize("theta", [0.2, 0.45, 0.57])
def test_walk_equals_characterisation(n, n_leaf, n_group, seed, theta):
    pos, m = W.plummer_clumps(n, seed, n_clumps=6)
    O = oracle.Tree(pos, m, n_leaf, n_group)
    com = _com32(O)
    for a, b in zip(O.lists_com(theta, com), O.lists_com(theta, com, brute=True)):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("gen,seed", [("plummer", 7), ("clumps", 8), ("milky_way", 9)])
def test_cells_holding_group_particles_are_opened(gen, seed):
    n = 6000
    pos, m = {"plummer": lambda: W.plummer(n, seed),
              "clumps": lambda: W.plummer_clumps(n, seed, n_clumps=10),
              "milky_way": lambda: W.milky_way(n, seed)}[gen]()
    O = oracle.Tree(pos, m, 8, 32)
    ex = O.export()
    first, cnt = ex["topo"][:, 2].astype(np.int64), ex["topo"][:, 3].astype(np.int64)
    c_off, c_ids, _, _ = O.lists_com(0.57, _com32(O))
    for g, gc in enumerate(ex["groups"]):
        lo, hi = first[gc], first[gc] + cnt[gc]
        c = c_ids[c_off[g]:c_off[g + 1]]
        # a cell in the cell list shares no particle with the group
        assert np.all((first[c] + cnt[c] <= lo) | (first[c] >= hi)), g


def test_theta_zero_lists_give_the_direct_sum():
    pos, m = W.plummer(1500, 11)
    O = oracle.Tree(pos, m, 8, 32)
    lists = O.lists_com(0.0, _com32(O))
    a, p = O.forces_lists(lists, 0.01)
    ad, pd = oracle.direct(pos, m, 0.01)
    assert np.max(oracle.rel_err(a, ad)) < 1e-12 and np.max(oracle.rel_err(p, pd)) < 1e-12


def test_error_falls_with_theta():
    pos, m = W.plummer(4000, 12)
    O = oracle.Tree(pos, m, 16, 64)
    ad, _ = oracle.direct(pos, m, 0.01)
    med = []
    for th in (0.2, 0.35, 0.5):
        a, _ = O.forces_lists(O.lists_com(th, _com32(O)), 0.01)
        med.append(np.median(oracle.rel_err(a, ad)))
    assert med[0] < med[1] < med[2] < 1e-2
