"""The force entry point for callers that cannot allocate
(octgrav_forces_noalloc) against octgrav_forces: same outputs bit for bit,
same interaction totals and FP64 diagnostics, on two calls in a row whose
second tree is smaller (the scratch array keeps the first call's contents),
with every library allocation made to fail while it runs."""
import numpy as np
import pytest

from paper_1005_5384_amd import octgrav as og
from paper_1005_5384_amd import workloads as W

pytestmark = pytest.mark.gpu


def _compare(T, theta, eps, monkeypatch):
    import torch
    a_ref, p_ref = T.forces(theta, eps)
    torch.cuda.synchronize()
    a_ref, p_ref = a_ref.cpu().numpy(), p_ref.cpu().numpy()
    c_ref = T.last_counts()
    d_ref = T.diagnostics()
    acc = torch.full((T.n, 3), float("nan"), dtype=torch.float32, device="cuda")
    pot = torch.full((T.n,), float("nan"), dtype=torch.float32, device="cuda")
    monkeypatch.setenv("OCTGRAV_FAIL_ALLOC", "1")
    try:
        T.forces_noalloc(theta, eps, acc, pot)
        torch.cuda.synchronize()
    finally:
        monkeypatch.delenv("OCTGRAV_FAIL_ALLOC")
    a, p = acc.cpu().numpy(), pot.cpu().numpy()
    print(f"n={T.n} theta={theta}: acc bit-equal {np.array_equal(a, a_ref)}, "
          f"pot bit-equal {np.array_equal(p, p_ref)}", flush=True)
    assert np.array_equal(a, a_ref) and np.array_equal(p, p_ref)
    assert T.last_counts() == c_ref
    mom, w = T.diagnostics()
    assert np.array_equal(mom, d_ref[0]) and w == d_ref[1]


def test_noalloc_equals_forces_on_two_calls(monkeypatch):
    import torch
    assert torch.cuda.is_available()
    big = W.WORKLOADS["plummer1m"]
    pos, m = W.make("plummer1m")
    T1 = og.Tree(pos, m, big["n_leaf"], 64)
    _compare(T1, 0.5, big["eps"], monkeypatch)        # fused wave path
    small = W.WORKLOADS["plummer16k"]
    pos, m = W.make("plummer16k")
    T2 = og.Tree(pos, m, small["n_leaf"], 64)
    _compare(T2, 0.3, small["eps"], monkeypatch)      # smaller tree, small angle
    _compare(T2, 0.75, small["eps"], monkeypatch)
    # frontier overflows into the global-memory queues held in the scratch
    monkeypatch.setenv("OCTGRAV_LDS_QUEUE", "64")
    T3 = og.Tree(pos, m, small["n_leaf"], 64)
    monkeypatch.delenv("OCTGRAV_LDS_QUEUE")
    _compare(T3, 0.5, small["eps"], monkeypatch)


def test_noalloc_learned_and_limits(monkeypatch):
    import torch
    from paper_1005_5384_amd import learned as L
    w = W.WORKLOADS["plummer16k"]
    pos, m = W.make("plummer16k")
    T = og.Tree(pos, m, w["n_leaf"], 64)
    net = og.Mlp(L.load_params())
    T.set_mac(net, 0.4, 0.8, 4.21e-4, 30 * 4.21e-4)
    try:
        _compare(T, 0.5625, w["eps"], monkeypatch)
        assert T.mac_stats()["band"] > 0
    finally:
        T.set_mac(None)
    acc = torch.empty((T.n, 3), dtype=torch.float32, device="cuda")
    monkeypatch.setenv("OCTGRAV_NOALLOC_LIMIT", "4096")
    with pytest.raises(og.OctgravError, match="scratch"):
        T.forces_noalloc(0.5, w["eps"], acc)
    monkeypatch.delenv("OCTGRAV_NOALLOC_LIMIT")
    for bad in ((1.5, w["eps"]), (0.5, 0.0)):
        with pytest.raises(og.OctgravError):
            T.forces_noalloc(*bad, acc)
