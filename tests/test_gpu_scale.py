"""Parity at the largest workload (16M-particle heterogeneous galaxy mix,
n_leaf 32) in the launch configuration the benchmark uses, on sampled
groups the oracle evaluates one by one."""
import numpy as np
import pytest

import oracle
from paper_1005_5384_amd import octgrav as og
from paper_1005_5384_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def galaxy():
    import torch
    assert torch.cuda.is_available()
    w = W.WORKLOADS["galaxy16m"]
    print("galaxy16m: generating", flush=True)
    pos, m = W.make("galaxy16m")
    print("galaxy16m: GPU tree", flush=True)
    T = og.Tree(pos, m, w["n_leaf"], 64)
    print("galaxy16m: oracle tree", flush=True)
    R = oracle.Tree(pos, m, w["n_leaf"], 64)
    return pos, m, w, T, R


@pytest.mark.parametrize("theta", [0.5])
def test_galaxy16m_sampled_groups_match_oracle(galaxy, theta):
    pos, m, w, T, R = galaxy
    assert T.stats["n_groups"] == R.n_groups
    acc, pot = T.forces(theta, w["eps"])
    a = acc.cpu().numpy().astype(np.float64)
    p = pot.cpu().numpy().astype(np.float64)
    sel = np.sort(np.random.default_rng(16).choice(R.n_groups, 96, replace=False))
    ra, rp = R.forces(theta, w["eps"], groups=sel)
    k = ~np.isnan(rp)
    assert k.sum() > 96
    ea = oracle.rel_err(a[k], ra[k])
    ep = np.abs(p[k] - rp[k]) / np.abs(rp[k])
    assert np.median(ea) < 1e-5 and ea.max() < 1e-4, (np.median(ea), ea.max())
    assert np.median(ep) < 1e-5 and ep.max() < 1e-4, (np.median(ep), ep.max())
    # momentum and energy diagnostics of the whole call against FP64 sums of the outputs
    mom, wsum = T.diagnostics()
    md, wd = oracle.diagnostics(m, a, p)
    np.testing.assert_allclose(mom, md, rtol=1e-9, atol=1e-12)
    assert abs(wsum - wd) <= 1e-9 * abs(wd)


def test_galaxy16m_learned_runs_with_fallback_guard(galaxy):
    # The trained network on an out-of-distribution workload: the call
    # completes, forces stay close to the theta path's, and a budget of zero
    # sends every group that accepted a band cell back to theta.
    from paper_1005_5384_amd import learned as L
    pos, m, w, T, R = galaxy
    net = og.Mlp(L.load_params())
    ref, _ = T.forces(0.5, w["eps"])
    try:
        T.set_mac(net, 0.4, 0.8, 3.57e-4, 30 * 3.57e-4)
        acc, _ = T.forces(0.5, w["eps"])
        st = T.mac_stats()
        assert st["band"] > 0
        e = (acc - ref).norm(dim=1) / ref.norm(dim=1)
        assert float(e.median()) < 2e-3
        T.set_mac(net, 0.4, 0.8, 3.57e-4, 0.0)
        acc0, _ = T.forces(0.5, w["eps"])
        assert T.mac_stats()["fell_back"] > 0
    finally:
        T.set_mac(None)
