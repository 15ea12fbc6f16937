"""The experiment configurations on the GPU: the Milky-Way-like stand-in
through the default path (lists bit-exact, forces within the gates of the
same-tree FP64 oracle, per-particle walk included), and the sweep driver
end to end on a small workload."""
import io
import json

import numpy as np
import pytest

import oracle
from paper_1005_5384_amd import experiments as X
from paper_1005_5384_amd import octgrav as og
from paper_1005_5384_amd import workloads as W

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    assert torch.cuda.is_available()
    return torch


@pytest.mark.parametrize("n_leaf,n_group", [(16, 64), (16, 1), (4, 256)])
def test_milky_way_parity(n_leaf, n_group):
    torch = _torch()
    pos, m = W.milky_way(12000, 109)
    T = og.Tree(pos, m, n_leaf, n_group, device_build=True)
    O = oracle.Tree(pos, m, n_leaf, n_group)
    for theta in (0.3, 0.7):
        for a, b in zip(T.lists(theta), O.lists(theta)):
            assert np.array_equal(a, b)
        acc, pot = T.forces(theta, 1e-3)
        torch.cuda.synchronize()
        ar, pr = O.forces(theta, 1e-3)
        ea = oracle.rel_err(acc.double().cpu().numpy(), ar)
        ep = oracle.rel_err(pot.double().cpu().numpy(), pr)
        assert np.median(ea) <= 1e-5 and ea.max() <= 1e-4, (theta, ea.max())
        assert np.median(ep) <= 1e-5 and ep.max() <= 1e-4, (theta, ep.max())


def test_sweep_driver_small():
    _torch()
    buf = io.StringIO()
    rows = X.leaf_group_sweep("plummer16k", 0.5, leaves=(8, 16), groups=(1, 64), steps=2, out=buf,
                             extra=())
    lines = [json.loads(s) for s in buf.getvalue().splitlines()]
    assert len(rows) == 4 and lines == rows
    for r in rows:
        assert r["ms"] > 0 and 0 < r["err"]["median"] <= r["err"]["p99"] <= r["err"]["max"] < 0.05
    # groups of one particle walk per particle: no more interactions than groups of 64
    # (a group's walk is conservative for every member)
    one = {r["n_leaf"]: r for r in rows if r["n_group"] == 1}
    g64 = {r["n_leaf"]: r for r in rows if r["n_group"] == 64}
    for nl in (8, 16):
        assert one[nl]["pc_per_particle"] + one[nl]["pp_per_particle"] <= \
            g64[nl]["pc_per_particle"] + g64[nl]["pp_per_particle"]
