"""Seeded random configurations through every walk: particle counts from 1
to 6000 in Plummer, clumped, Milky-Way-like and lattice (plane ties,
coincident points) layouts, random leaf and group capacities and opening
angles.  Lists of the three paths, of the device-built tree and of the
offset test must equal the oracle's bit for bit, and forces must meet the
gates of the same-tree FP64 oracle."""
import numpy as np
import pytest

import oracle
from paper_1005_5384_amd import octgrav as og
from paper_1005_5384_amd import workloads as W

pytestmark = pytest.mark.gpu


def _case(k):
    rng = np.random.default_rng(1000 + k)
    n = int(rng.choice([1, 2, 3, 7, 64, 65, 500, 1999, 4096, 6000]))
    kind = ["plummer", "clumps", "milky_way", "lattice"][k % 4]
    if kind == "plummer":
        pos, m = W.plummer(n, 2000 + k)
    elif kind == "clumps":
        pos, m = W.plummer_clumps(n, 2000 + k, n_clumps=5)
    elif kind == "milky_way":
        pos, m = W.milky_way(n, 2000 + k)
    else:
        pos = (rng.integers(-3, 4, (n, 3)) * 0.5).astype(np.float32)
        m = rng.uniform(0.5, 2.0, n).astype(np.float32)
    n_leaf = int(rng.choice([1, 2, 8, 16, 33, 64]))
    n_group = int(rng.choice([1, 5, 16, 64, 100, 1024]))
    theta = float(rng.choice([0.0, 0.2, 0.35, 0.41, 0.5, 0.57, 0.8, 1.0]))
    return pos, m, n_leaf, n_group, theta


@pytest.mark.parametrize("k", range(32))
def test_random_configuration(k):
    import torch
    assert torch.cuda.is_available()
    pos, m, n_leaf, n_group, theta = _case(k)
    O = oracle.Tree(pos, m, n_leaf, n_group)
    ref = O.lists(theta)
    for dev in (False, True):
        T = og.Tree(pos, m, n_leaf, n_group, device_build=dev)
        for path in (None, "two_pass", "fused_block", "fused_wave"):
            for a, b in zip(T.lists(theta, path=path), ref):
                assert np.array_equal(a, b), (k, dev, path)
        if theta <= 0.57:
            com = T.export()["mp"][:, :3]
            for a, b in zip(T.lists(theta, com=True), O.lists_com(theta, com)):
                assert np.array_equal(a, b), (k, dev, "com")
        acc, pot = T.forces(theta, 0.01)
        torch.cuda.synchronize()
        ar, pr = O.forces(theta, 0.01)
        a, p = acc.double().cpu().numpy(), pot.double().cpu().numpy()
        if pos.shape[0] > 1:
            na = np.linalg.norm(ar, axis=1)
            keep = na >= 1e-6 * np.median(na)
            ea = oracle.rel_err(a[keep], ar[keep])
            ep = oracle.rel_err(p, pr)
            assert np.median(ea) <= 1e-5 and ea.max() <= 1e-4, (k, dev, ea.max())
            assert np.median(ep) <= 1e-5 and ep.max() <= 1e-4, (k, dev, ep.max())
        else:
            assert np.all(a == 0) and np.all(p == 0)
        T.close()


@pytest.mark.parametrize("k", range(10))
def test_random_learned_configuration(k):
    """The learned criterion on seeded random trees, bands, tau_pair and
    budgets: the walk's exported decisions replayed by the oracle give the
    same lists and the same fall-backs, and the forces of those lists meet
    the gates of the oracle's FP64 evaluation."""
    import torch
    assert torch.cuda.is_available()
    from paper_1005_5384_amd import learned as L
    rng = np.random.default_rng(3000 + k)
    pos, m, n_leaf, n_group, _ = _case(k)
    lo = float(rng.choice([0.3, 0.4, 0.5]))
    hi = lo + float(rng.choice([0.2, 0.3, 0.45]))
    theta = float(rng.choice([0.4, 0.55, 0.7]))
    tau = float(10.0 ** rng.uniform(-5, -2))
    budget = float(rng.choice([-1.0, 3 * tau, 30 * tau, 1e9]))
    T = og.Tree(pos, m, n_leaf, n_group, device_build=bool(k % 2))
    O = oracle.Tree(pos, m, n_leaf, n_group)
    T.set_mac(og.Mlp(L.load_params()), lo, hi, tau, budget)
    off, cells, scores, fb = T.mac_trace(theta)
    g = np.repeat(np.arange(off.size - 1, dtype=np.int32), np.diff(off))
    ref, rfb = O.lists_learned(theta, lo, hi, oracle.log10_threshold(tau), budget,
                               replay=(g, cells, scores))
    got = T.lists(theta)
    for a, b in zip(got, ref):
        assert np.array_equal(a, b), k
    assert np.array_equal(fb, rfb), k
    if budget < 0:
        assert np.all(fb == 1) or fb.size == 0
    acc, pot = T.forces(theta, 0.01)
    torch.cuda.synchronize()
    ar, pr = O.forces_lists(ref, 0.01)
    if pos.shape[0] > 1:
        na = np.linalg.norm(ar, axis=1)
        keep = na >= 1e-6 * np.median(na)
        ea = oracle.rel_err(acc.double().cpu().numpy()[keep], ar[keep])
        ep = oracle.rel_err(pot.double().cpu().numpy(), pr)
        assert np.median(ea) <= 1e-5 and ea.max() <= 1e-4, (k, ea.max())
        assert np.median(ep) <= 1e-5 and ep.max() <= 1e-4, (k, ep.max())
    T.set_mac(None)
    T.close()
