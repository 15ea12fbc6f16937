"""Pins of the oracle's leapfrog: time reversibility, second-order
convergence on a circular binary, bounded energy error, and the Plummer
equilibrium sampler's virial ratio."""
import numpy as np

import oracle
from paper_1005_5384_amd import workloads as W


def _binary():
    # equal masses 1/2 at +-1/2 on x, circular: omega^2 = M / d^3 = 1, speed 1/2
    pos = np.array([[-0.5, 0, 0], [0.5, 0, 0]])
    vel = np.array([[0, -0.5, 0], [0, 0.5, 0]])
    return pos, vel, np.array([0.5, 0.5])


def test_time_reversible():
    rng = np.random.default_rng(1)
    pos, vel = rng.normal(0, 1, (20, 3)), rng.normal(0, 0.3, (20, 3))
    m = rng.uniform(0.5, 1.5, 20) / 20
    p1, v1, _ = oracle.leapfrog(pos, vel, m, 0.05, 0.01, 50)
    p0, v0, _ = oracle.leapfrog(p1, v1, m, 0.05, -0.01, 50)
    np.testing.assert_allclose(p0, pos, atol=1e-11)
    np.testing.assert_allclose(v0, vel, atol=1e-11)


def test_binary_second_order_after_one_period():
    pos, vel, m = _binary()
    errs = []
    for k in (200, 400, 800):
        p, _, _ = oracle.leapfrog(pos, vel, m, 1e-7, 2 * np.pi / k, k)
        errs.append(np.abs(p - pos).max())
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.6 < r1 < 4.4 and 3.6 < r2 < 4.4, (errs, r1, r2)


def test_binary_energy_bounded():
    pos, vel, m = _binary()
    _, _, en = oracle.leapfrog(pos, vel, m, 1e-7, 2 * np.pi / 400, 4000)
    E = en.sum(1)
    np.testing.assert_allclose(en[0], [0.125, -0.25], rtol=1e-9)
    assert np.abs(E - E[0]).max() < 1e-4 * abs(E[0])


def test_plummer_sampler_virial():
    pos, vel, m = W.plummer_with_velocities(4096, 7)
    _, _, en = oracle.leapfrog(pos, vel, m, 1e-4, 0.0, 0)
    K, Wp = en[0]
    assert abs(2 * K / abs(Wp) - 1) < 0.06, 2 * K / abs(Wp)   # virial equilibrium
    assert abs(Wp + 3 * np.pi / 32) < 0.03                      # W = -3 pi / 32 for a = 1
