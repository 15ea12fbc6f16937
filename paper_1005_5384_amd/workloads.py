"""Seeded synthetic particle distributions.

This module only draws random numbers: it holds no part of the tree-code's
arithmetic, so both the HIP path and the CPU oracle can be fed from it.
Every generator works in float64 with numpy's PCG64 and rounds once to
float32 at the end.  Masses are equal (1/N) unless stated.

The paper measures on a Milky Way galaxy model (Section 3, bulge:disk:halo
mass 1:1:4) whose generator is not available; the distributions below stand
in for it with the same structural ingredients: a centrally concentrated
spheroid (Plummer / Hernquist), a thin exponential disc and dense clumps.
"""
from __future__ import annotations

import numpy as np

PLUMMER_RCUT = 22.8


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


def _isotropic(rng: np.random.Generator, r: np.ndarray) -> np.ndarray:
    """Points at radii r with isotropic directions (float64, shape [n,3])."""
    n = r.shape[0]
    cth = rng.uniform(-1.0, 1.0, n)
    phi = rng.uniform(0.0, 2.0 * np.pi, n)
    sth = np.sqrt(np.maximum(0.0, 1.0 - cth * cth))
    return np.stack([r * sth * np.cos(phi), r * sth * np.sin(phi), r * cth], axis=1)


def _radii(rng: np.random.Generator, n: int, inverse_cdf, rcut: float) -> np.ndarray:
    """Draw n radii by inverse-CDF sampling, redrawing those beyond rcut."""
    out = np.empty(n)
    todo = np.arange(n)
    while todo.size:
        x = rng.uniform(0.0, 1.0, todo.size)
        r = inverse_cdf(x)
        ok = np.isfinite(r) & (r <= rcut)
        out[todo[ok]] = r[ok]
        todo = todo[~ok]
    return out


def plummer_radii(rng: np.random.Generator, n: int, a: float = 1.0,
                  rcut: float = PLUMMER_RCUT) -> np.ndarray:
    # Plummer enclosed-mass fraction X = r^3/(r^2+a^2)^{3/2}, inverted.
    def inv(x):
        with np.errstate(divide="ignore", invalid="ignore"):
            return a / np.sqrt(x ** (-2.0 / 3.0) - 1.0)
    return _radii(rng, n, inv, rcut * a)


def plummer(n: int, seed: int, a: float = 1.0, rcut: float = PLUMMER_RCUT):
    """Plummer sphere (scale radius a, truncated at rcut*a), equal masses 1/n."""
    rng = _rng(seed)
    r = plummer_radii(rng, n, a, rcut)
    pos = _isotropic(rng, r)
    return pos.astype(np.float32), np.full(n, 1.0 / n, dtype=np.float32)


def _plummer_phase(rng: np.random.Generator, n: int, rcut: float):
    """FP64 positions and velocities of a Plummer sphere (a = 1, G = 1, total
    mass 1) in equilibrium: radii as `plummer`, isotropic speeds
    v = q v_esc(r), v_esc = sqrt(2) (1 + r^2)^-1/4, with q drawn from
    g(q) ~ q^2 (1 - q^2)^(7/2) by rejection (Aarseth, Henon & Wielen 1974)."""
    r = plummer_radii(rng, n, 1.0, rcut)
    pos = _isotropic(rng, r)
    q = np.empty(n)
    todo = np.arange(n)
    while todo.size:
        x = rng.uniform(0.0, 1.0, todo.size)
        y = rng.uniform(0.0, 0.1, todo.size)
        ok = y < x * x * (1.0 - x * x) ** 3.5
        q[todo[ok]] = x[ok]
        todo = todo[~ok]
    v = q * np.sqrt(2.0) * (1.0 + r * r) ** -0.25
    return pos, _isotropic(rng, v)


def plummer_with_velocities(n: int, seed: int, rcut: float = PLUMMER_RCUT):
    """Plummer sphere (a = 1, G = 1, total mass 1) in equilibrium (see
    `_plummer_phase`).  Returns float32 (pos, vel, mass)."""
    pos, vel = _plummer_phase(_rng(seed), n, rcut)
    return pos.astype(np.float32), vel.astype(np.float32), np.full(n, 1.0 / n, dtype=np.float32)


def plummer_pair_orbit(n: int, seed: int, separation: float = 8.0, impact: float = 1.0,
                       rcut: float = PLUMMER_RCUT):
    """Initial conditions of a two-Plummer merger: two equilibrium spheres
    (a = 1, half the particles and about half the mass each, internal speeds
    scaled by sqrt(1/2) for that mass) whose centres are (separation, impact,
    0) apart and approach along x at the parabolic relative speed
    sqrt(2 G M_tot / r0), M_tot = 1.  The centre of mass is at rest at the
    origin.  Returns float32 (pos, vel, mass)."""
    rng = _rng(seed)
    h = n // 2
    pa, va = _plummer_phase(rng, h, rcut)
    pb, vb = _plummer_phase(rng, n - h, rcut)
    va *= np.sqrt(0.5)
    vb *= np.sqrt(0.5)
    r0 = np.array([separation, impact, 0.0])
    v = np.sqrt(2.0 / np.linalg.norm(r0))
    fa, fb = (n - h) / n, h / n  # each centre's share of the relative vector
    pa += fa * r0
    pb -= fb * r0
    va[:, 0] -= fa * v
    vb[:, 0] += fb * v
    pos = np.concatenate([pa, pb])
    vel = np.concatenate([va, vb])
    return pos.astype(np.float32), vel.astype(np.float32), np.full(n, 1.0 / n, dtype=np.float32)


def two_plummer(n: int, seed: int, separation: float):
    """Two equal Plummer spheres (a = 1) whose centres are `separation` apart on x."""
    rng = _rng(seed)
    h = n // 2
    pa = _isotropic(rng, plummer_radii(rng, h))
    pb = _isotropic(rng, plummer_radii(rng, n - h))
    pa[:, 0] -= 0.5 * separation
    pb[:, 0] += 0.5 * separation
    pos = np.concatenate([pa, pb])
    return pos.astype(np.float32), np.full(n, 1.0 / n, dtype=np.float32)


def _largest_remainder(weights: np.ndarray, n: int) -> np.ndarray:
    q = weights / weights.sum() * n
    base = np.floor(q).astype(np.int64)
    rem = n - int(base.sum())
    order = np.argsort(-(q - base), kind="stable")
    base[order[:rem]] += 1
    return base


def plummer_clumps(n: int, seed: int, n_clumps: int = 64, sigma: float = 1.0,
                   rmin: float = 0.01, rmax: float = 0.1):
    """Clustered mix: Plummer clumps with log-normal masses, scale radii
    U[rmin, rmax], centres uniform in the unit cube, each cut at 22.8 scale
    radii.  Particle counts are proportional to clump mass."""
    rng = _rng(seed)
    cm = rng.lognormal(0.0, sigma, n_clumps)
    counts = _largest_remainder(cm, n)
    radii = rng.uniform(rmin, rmax, n_clumps)
    centres = rng.uniform(0.0, 1.0, (n_clumps, 3))
    parts = []
    for k in range(n_clumps):
        if counts[k] == 0:
            continue
        p = _isotropic(rng, plummer_radii(rng, int(counts[k]), radii[k]))
        parts.append(p + centres[k])
    pos = np.concatenate(parts)
    return pos.astype(np.float32), np.full(n, 1.0 / n, dtype=np.float32)


def galaxy_mix(n: int, seed: int, n_clumps: int = 256):
    """Heterogeneous galaxy-like mix: 40% Hernquist halo (a = 1, cut 100a),
    50% exponential disc (R_d = 0.3 cut 10 R_d, sech^2 with z_d = 0.03 cut
    10 z_d), 10% dense Plummer clumps (equal counts, scale radii
    U[0.005, 0.02], centres drawn from the disc)."""
    rng = _rng(seed)
    n_halo = int(round(0.4 * n))
    n_disc = int(round(0.5 * n))
    n_clump = n - n_halo - n_disc

    def hern_inv(x):
        s = np.sqrt(x)
        with np.errstate(divide="ignore"):
            return s / (1.0 - s)
    halo = _isotropic(rng, _radii(rng, n_halo, hern_inv, 100.0))

    def disc_points(m):
        rd, zd = 0.3, 0.03
        R = np.empty(m)
        todo = np.arange(m)
        while todo.size:
            v = rng.gamma(2.0, rd, todo.size)
            ok = v <= 10 * rd
            R[todo[ok]] = v[ok]
            todo = todo[~ok]
        z = np.empty(m)
        todo = np.arange(m)
        while todo.size:
            u = rng.uniform(0.0, 1.0, todo.size)
            with np.errstate(divide="ignore"):
                v = zd * np.arctanh(2.0 * u - 1.0)
            ok = np.isfinite(v) & (np.abs(v) <= 10 * zd)
            z[todo[ok]] = v[ok]
            todo = todo[~ok]
        ph = rng.uniform(0.0, 2.0 * np.pi, m)
        return np.stack([R * np.cos(ph), R * np.sin(ph), z], axis=1)

    disc = disc_points(n_disc)
    centres = disc_points(n_clumps)
    counts = _largest_remainder(np.ones(n_clumps), n_clump)
    radii = rng.uniform(0.005, 0.02, n_clumps)
    cl = [_isotropic(rng, plummer_radii(rng, int(counts[k]), radii[k])) + centres[k]
          for k in range(n_clumps) if counts[k] > 0]
    pos = np.concatenate([halo, disc] + cl)
    return pos.astype(np.float32), np.full(n, 1.0 / n, dtype=np.float32)


def _hernquist_radii(rng: np.random.Generator, n: int, a: float, rcut: float) -> np.ndarray:
    """Hernquist radii: M(<r)/M = (r / (r + a))^2, so r = a sqrt(X) / (1 - sqrt(X))."""
    def inv(x):
        s = np.sqrt(x)
        with np.errstate(divide="ignore"):
            return a * s / (1.0 - s)
    return _radii(rng, n, inv, rcut)


def _exp_disc(rng: np.random.Generator, m: int, rd: float, zd: float) -> np.ndarray:
    """Exponential disc: R ~ Gamma(2, rd) cut at 10 rd, sech^2 vertical profile
    z = zd atanh(2U - 1) cut at 10 zd, uniform azimuth."""
    R = np.empty(m)
    todo = np.arange(m)
    while todo.size:
        v = rng.gamma(2.0, rd, todo.size)
        ok = v <= 10 * rd
        R[todo[ok]] = v[ok]
        todo = todo[~ok]
    z = np.empty(m)
    todo = np.arange(m)
    while todo.size:
        u = rng.uniform(0.0, 1.0, todo.size)
        with np.errstate(divide="ignore"):
            v = zd * np.arctanh(2.0 * u - 1.0)
        ok = np.isfinite(v) & (np.abs(v) <= 10 * zd)
        z[todo[ok]] = v[ok]
        todo = todo[~ok]
    ph = rng.uniform(0.0, 2.0 * np.pi, m)
    return np.stack([R * np.cos(ph), R * np.sin(ph), z], axis=1)


# Component fractions of the Milky-Way-like stand-in: bulge : disc : halo =
# 1 : 1 : 4 by mass, the proportions of the paper's galaxy model (Sec. 3).
MW_FRACTIONS = (1.0 / 6.0, 1.0 / 6.0, 4.0 / 6.0)


def milky_way(n: int, seed: int):
    """Milky-Way-like stand-in with equal-mass particles: a Hernquist bulge
    (a = 0.1, cut 30a), an exponential disc (R_d = 0.3, z_d = 0.03) and a
    Hernquist halo (a = 1, cut 100a) holding 1/6, 1/6 and 4/6 of the particles
    (largest-remainder counts)."""
    rng = _rng(seed)
    nb, nd, nh = _largest_remainder(np.array(MW_FRACTIONS), n)
    bulge = _isotropic(rng, _hernquist_radii(rng, int(nb), 0.1, 3.0))
    disc = _exp_disc(rng, int(nd), 0.3, 0.03)
    halo = _isotropic(rng, _hernquist_radii(rng, int(nh), 1.0, 100.0))
    pos = np.concatenate([bulge, disc, halo])
    return pos.astype(np.float32), np.full(n, 1.0 / n, dtype=np.float32)


def sample_indices(n: int, k: int, seed: int) -> np.ndarray:
    """k distinct particle indices drawn without replacement (sorted, int64)."""
    rng = _rng(seed)
    k = min(k, n)
    return np.sort(rng.choice(n, size=k, replace=False)).astype(np.int64)


# Named workloads: (generator, kwargs, n, eps, n_leaf, theta list).
WORKLOADS = {
    "plummer16k": dict(gen="plummer", n=16384, seed=101, eps=0.01, n_leaf=16, thetas=(0.5,)),
    "plummer1m": dict(gen="plummer", n=1 << 20, seed=102, eps=1e-3, n_leaf=16,
                      thetas=(0.3, 0.5, 0.75), sample=4096, sample_seed=4096),
    "clumps4m": dict(gen="plummer_clumps", n=1 << 22, seed=103, eps=1e-3, n_leaf=32,
                     thetas=(0.5,), sample=4096, sample_seed=4096),
    "galaxy16m": dict(gen="galaxy_mix", n=1 << 24, seed=108, eps=5e-4, n_leaf=32,
                      thetas=(0.5,), sample=4096, sample_seed=4096),
    "milkyway1m": dict(gen="milky_way", n=1 << 20, seed=109, eps=1e-3, n_leaf=16,
                       thetas=(0.5,), sample=4096, sample_seed=4096),
}


# Training sets of the learned acceptance criterion: a Plummer sphere and
# static two-Plummer configurations at three separations (scale radii), all
# 2^18 particles, softened as the 2^20 Plummer workload.
TRAINING_SETS = (
    dict(gen="plummer", n=1 << 18, seed=104),
    dict(gen="two_plummer", n=1 << 18, seed=105, separation=2.0),
    dict(gen="two_plummer", n=1 << 18, seed=106, separation=4.0),
    dict(gen="two_plummer", n=1 << 18, seed=107, separation=8.0),
)
TRAINING_EPS = 1e-3

# Snapshots of a dynamic two-Plummer merger (the library's leapfrog, tree
# rebuilt on the GPU every step) join the static sets: 2^18 particles,
# centres 8 apart with impact parameter 1 on a parabolic orbit, dt = 1/64,
# a snapshot every 256 steps (4 time units), five snapshots from t = 0 to 16.
MERGER_SET = dict(n=1 << 18, seed=110, separation=8.0, impact=1.0, dt=1.0 / 64, every=256,
                  count=5, theta=0.5)


def make_training(k: int):
    """Positions and masses of training set k."""
    w = dict(TRAINING_SETS[k])
    gen = {"plummer": plummer, "two_plummer": two_plummer}[w.pop("gen")]
    n, seed = w.pop("n"), w.pop("seed")
    return gen(n, seed, **w)


def make(name: str, n: int | None = None):
    """Positions [n,3] f32 and masses [n] f32 of a named workload."""
    w = WORKLOADS[name]
    n = w["n"] if n is None else n
    gen = {"plummer": plummer, "plummer_clumps": plummer_clumps, "galaxy_mix": galaxy_mix,
           "milky_way": milky_way}[w["gen"]]
    return gen(n, w["seed"])
