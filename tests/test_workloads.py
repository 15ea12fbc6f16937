"""Input generators against the closed forms of their distributions: the
Milky-Way-like 1:1:4 stand-in's component counts and Hernquist medians, the
disc's cuts, seeding."""
import numpy as np

from paper_1005_5384_amd import workloads as W


def _hernquist_median(a, rcut):
    # M(<r) = (r / (r + a))^2 truncated at rcut: median where M(<r) = M(<rcut) / 2
    s = np.sqrt(0.5 * (rcut / (rcut + a)) ** 2)
    return a * s / (1 - s)


def test_milky_way_components():
    n = 120001
    pos, m = W.milky_way(n, 3)
    assert pos.shape == (n, 3) and pos.dtype == np.float32 and np.all(m == np.float32(1 / n))
    nb, nd, nh = W._largest_remainder(np.array(W.MW_FRACTIONS), n)
    assert nb + nd + nh == n and abs(nh - 4 * nb) <= 4 and abs(nb - nd) <= 1
    r = np.linalg.norm(pos.astype(np.float64), axis=1)
    bulge, disc, halo = pos[:nb], pos[nb:nb + nd], r[nb + nd:]
    rb = np.linalg.norm(bulge.astype(np.float64), axis=1)
    assert rb.max() <= 3.0 and halo.max() <= 100.0
    np.testing.assert_allclose(np.median(rb), _hernquist_median(0.1, 3.0), rtol=0.03)
    np.testing.assert_allclose(np.median(halo), _hernquist_median(1.0, 100.0), rtol=0.03)
    R = np.hypot(disc[:, 0], disc[:, 1])
    assert R.max() <= 3.0 + 1e-6 and np.abs(disc[:, 2]).max() <= 0.3 + 1e-6
    # Gamma(2, 0.3) truncated at 3: mean radius close to 2 R_d
    np.testing.assert_allclose(R.mean(), 0.6, rtol=0.03)


def test_milky_way_seeded():
    a, _ = W.milky_way(5000, 7)
    b, _ = W.milky_way(5000, 7)
    c, _ = W.milky_way(5000, 8)
    assert np.array_equal(a, b) and not np.array_equal(a, c)


def test_nearest_rank():
    from paper_1005_5384_amd.experiments import nearest_rank
    x = np.array([5.0, 1.0, 4.0, 2.0, 3.0])
    assert nearest_rank(x, 0.5) == 3.0 and nearest_rank(x, 1.0) == 5.0
    assert nearest_rank(x, 0.2) == 1.0 and nearest_rank(x, 0.21) == 2.0
    y = np.arange(1, 101, dtype=float)
    assert nearest_rank(y, 0.99) == 99.0 and nearest_rank(y, 0.9) == 90.0


def test_plummer_pair_orbit():
    n = 20001
    pos, vel, m = W.plummer_pair_orbit(n, 4, separation=8.0, impact=1.0)
    h = n // 2
    p, v = pos.astype(np.float64), vel.astype(np.float64)
    mom = (m[:, None].astype(np.float64) * v).sum(0)
    assert np.abs(mom).max() < 5e-3                      # centre of mass at rest (sampling noise)
    ca, cb = p[:h].mean(0), p[h:].mean(0)
    np.testing.assert_allclose(ca - cb, [8.0, 1.0, 0.0], atol=0.15)
    va, vb = v[:h].mean(0), v[h:].mean(0)
    vpar = np.sqrt(2.0 / np.hypot(8.0, 1.0))            # parabolic: relative kinetic = potential
    np.testing.assert_allclose(va - vb, [-vpar, 0.0, 0.0], atol=0.01)
    # internal speeds scaled by sqrt(1/2) for half the mass: half the mean squared speed
    da = ((v[:h] - va) ** 2).sum(1).mean()
    _, v1, _ = W.plummer_with_velocities(h, 4)
    np.testing.assert_allclose(da, 0.5 * (v1.astype(np.float64) ** 2).sum(1).mean(), rtol=0.05)
