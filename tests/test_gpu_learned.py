"""GPU parity of the learned acceptance criterion (through the C ABI) against
the FP64 oracle: the network's forward pass, gradient and Adam step, the
learned walk's lists (replayed bit-exactly from the exported decisions), its
reductions to the theta walk, the group budget's fall-back, and the forces
under the learned lists."""
import numpy as np
import pytest

import oracle
from paper_1005_5384_amd import octgrav as og
from paper_1005_5384_amd import workloads as W

pytestmark = pytest.mark.gpu

NP = og.N_PARAMS
SPANS = {"W1": (0, 768), "b1": (768, 832), "W2": (832, 4928), "b2": (4928, 4992),
         "w3": (4992, 5056), "b3": (5056, 5057)}


def _torch():
    import torch
    assert torch.cuda.is_available()
    return torch


def _params(seed, scale=0.3):
    # FP32-representable parameters, so both sides start from the same values
    return np.random.default_rng(seed).normal(0, scale, NP).astype(np.float32)


def _close_scores(y, ref):
    # FP32 sums on the matrix cores vs FP64 sums: a hidden activation near a
    # BF16 rounding boundary can round the other way (about 1 sample in 300),
    # which moves the output by a BF16 step of one term.
    err = np.abs(y - ref) / (1.0 + np.abs(ref))
    assert np.quantile(err, 0.99) < 1e-5, np.quantile(err, 0.99)
    assert err.max() < 3e-2, err.max()


@pytest.mark.parametrize("b", [1, 63, 64, 1000])
def test_forward_matches_oracle(b):
    torch = _torch()
    rng = np.random.default_rng(b)
    P = _params(11, 0.25)
    x = rng.normal(0, 1, (b, 12)).astype(np.float32)
    m = og.Mlp(P)
    y = m.forward(torch.from_numpy(x).cuda()).cpu().numpy()
    _close_scores(y.astype(np.float64), oracle.mlp_forward(P.astype(np.float64), x))


def test_forward_single_unit_layout():
    # One nonzero path through the network pins the matrix-core operand
    # layout: y = w3[a] relu(W2[a, b] relu(W1[b, k] x_k + b1[b]) + b2[a]) + b3,
    # with every weight exact in BF16.
    torch = _torch()
    for a, b_, k in [(0, 0, 0), (5, 17, 3), (63, 40, 11), (33, 62, 7)]:
        P = np.zeros(NP, np.float32)
        P[0 + b_ * 12 + k] = 1.5
        P[768 + b_] = 0.25
        P[832 + a * 64 + b_] = -2.0
        P[4928 + a] = 4.0
        P[4992 + a] = 0.5
        P[5056] = 0.125
        x = np.zeros((64, 12), np.float32)
        x[:, k] = np.linspace(-1, 1, 64)
        y = og.Mlp(P).forward(torch.from_numpy(x).cuda()).cpu().numpy()
        ref = oracle.mlp_forward(P.astype(np.float64), x)
        plain = 0.5 * np.maximum(-2.0 * np.maximum(1.5 * x[:, k].astype(np.float64) + 0.25, 0) + 4.0,
                                 0) + 0.125
        np.testing.assert_allclose(ref, plain, atol=0.02)  # the formula, up to BF16 rounding
        np.testing.assert_allclose(y, ref, rtol=1e-6, atol=1e-6)


def test_loss_and_gradient_match_oracle():
    torch = _torch()
    rng = np.random.default_rng(3)
    P = _params(12, 0.2)
    x = rng.normal(0, 1, (777, 12)).astype(np.float32)
    t = rng.normal(-3, 1, 777).astype(np.float32)
    m = og.Mlp(P)
    loss, g = m.loss_grad(torch.from_numpy(x).cuda(), torch.from_numpy(t).cuda(), tau=0.9)
    rl, rg = oracle.mlp_loss_grad(P.astype(np.float64), x, t.astype(np.float64), tau=0.9)
    assert abs(loss - rl) <= 1e-5 * abs(rl)
    for name, (a, b) in SPANS.items():
        d = np.linalg.norm(g[a:b] - rg[a:b]) / np.linalg.norm(rg[a:b])
        assert d < 1e-3, (name, d)


def test_adam_matches_oracle():
    torch = _torch()
    rng = np.random.default_rng(4)
    P = _params(13, 0.2)
    x = rng.normal(0, 1, (256, 12)).astype(np.float32)
    t = rng.normal(-3, 1, 256).astype(np.float32)
    m = og.Mlp(P)
    _, g = m.loss_grad(torch.from_numpy(x).cuda(), torch.from_numpy(t).cuda())
    m.adam(1, lr=1e-3)
    m.adam(2, lr=1e-3)  # the same gradient again
    Pr, mr, vr = P.astype(np.float64), np.zeros(NP), np.zeros(NP)
    oracle.adam_step(Pr, mr, vr, g.astype(np.float64), 1, lr=1e-3)
    oracle.adam_step(Pr, mr, vr, g.astype(np.float64), 2, lr=1e-3)
    np.testing.assert_allclose(m.params(), Pr, rtol=0, atol=2e-6)
    # the inference image follows the new parameters
    y = m.forward(torch.from_numpy(x).cuda()).cpu().numpy()
    _close_scores(y.astype(np.float64), oracle.mlp_forward(m.params().astype(np.float64), x))


def test_training_reduces_loss():
    torch = _torch()
    rng = np.random.default_rng(5)
    x = rng.normal(0, 1, (4096, 12)).astype(np.float32)
    t = (-3 + x[:, 0] - 0.5 * x[:, 1] ** 2).astype(np.float32)
    m = og.Mlp(_params(14, 0.1))
    xd, td = torch.from_numpy(x).cuda(), torch.from_numpy(t).cuda()
    l0, _ = m.loss_grad(xd, td, want_grad=False)
    for s in range(1, 201):
        m.loss_grad(xd, td, want_grad=False)
        m.adam(s, lr=3e-3)
    l1, _ = m.loss_grad(xd, td, want_grad=False)
    assert l1 < 0.3 * l0, (l0, l1)


def test_training_resumed_from_checkpoint_equals_uninterrupted(tmp_path):
    """Two epochs, a checkpoint, a fresh network resumed from it for two more:
    parameters and Adam moments equal those of four uninterrupted epochs, bit
    for bit (the kernels and the batch order are deterministic)."""
    torch = _torch()
    from paper_1005_5384_amd import learned as L
    rng = np.random.default_rng(6)
    x = rng.normal(0, 1, (6000, 12)).astype(np.float32)
    t = (-3 + x[:, 0] - 0.5 * x[:, 1] ** 2).astype(np.float32)
    xd, td = torch.from_numpy(x).cuda(), torch.from_numpy(t).cuda()
    kw = dict(epochs=4, batch=1024, lr=3e-3, lr_final=3e-4, seed=7)
    full = L.train(xd, td, **kw)
    ck = str(tmp_path / "train.npz")
    L.train(xd, td, checkpoint=ck, stop_after=2, **kw)
    saved = L.load_checkpoint(ck)
    assert int(saved["epoch"]) == 2 and int(saved["step"]) == 2 * (6000 // 1024)
    resumed = L.train(xd, td, resume=ck, **kw)
    assert np.array_equal(full.params(), resumed.params())
    for a, b in zip(full.moments(), resumed.moments()):
        assert np.array_equal(a, b)
    # the resumed network differs from the two-epoch one (training went on)
    assert not np.array_equal(saved["params"], resumed.params())
    with pytest.raises(ValueError, match="settings"):
        L.train(xd, td, resume=ck, **dict(kw, lr=1e-3))


# ---------------------------------------------------------------- learned walk

@pytest.fixture(scope="module")
def setup():
    _torch()
    pos, m = W.plummer(8192, 51)
    T = og.Tree(pos, m, 16, 64)
    R = oracle.Tree(pos, m, 16, 64)
    P = _params(15, 0.1)
    net = og.Mlp(P)
    # a decision threshold in a wide gap between the scores near their median
    g, c = R.mac_band(0.3, 1.0)
    s = np.sort(oracle.mlp_forward(P.astype(np.float64), R.mac_features(g, c)))
    lo, hi = int(0.4 * s.size), int(0.6 * s.size)
    k = lo + int(np.argmax(np.diff(s[lo:hi])))
    ltau = 0.5 * (s[k] + s[k + 1])
    return pos, m, T, R, P, net, float(10.0 ** ltau)


def _replay(R, theta, tau, budget, off, cells, scores):
    g = np.repeat(np.arange(off.size - 1, dtype=np.int32), np.diff(off))
    return R.lists_learned(theta, 0.3, 1.0, oracle.log10_threshold(tau), budget,
                           replay=(g, cells, scores))


def _lists_equal(a, b):
    for name, x, y in zip(("c_off", "c_ids", "l_off", "l_ids"), a, b):
        assert x.shape == y.shape and np.array_equal(x, y), name


def test_learned_lists_replay_bit_exact(setup):
    pos, m, T, R, P, net, tau = setup
    T.set_mac(net, 0.3, 1.0, tau, float("inf"))
    try:
        off, cells, scores, fb = T.mac_trace(0.6)
        assert not fb.any() and cells.size > 0
        # scores: the network on the oracle's features of the same candidates
        g = np.repeat(np.arange(off.size - 1, dtype=np.int32), np.diff(off))
        _close_scores(scores.astype(np.float64),
                      oracle.mlp_forward(P.astype(np.float64), R.mac_features(g, cells)))
        ref, rfb = _replay(R, 0.6, tau, 1e30, off, cells, scores)
        assert not rfb.any()
        gl = T.lists(0.6)
        _lists_equal(gl, ref)
        # the decisions are mixed: some band cells accepted, some opened
        acc = scores <= np.float32(oracle.log10_threshold(tau))
        assert 0.2 < acc.mean() < 0.8
        st = T.mac_stats()
        assert st["band"] == cells.size and st["fell_back"] == 0
    finally:
        T.set_mac(None)


def test_learned_budget_fallback(setup):
    pos, m, T, R, P, net, tau = setup
    T.set_mac(net, 0.3, 1.0, tau, float("inf"))
    off, cells, scores, _ = T.mac_trace(0.6)
    lt = np.float32(oracle.log10_threshold(tau))
    # per-group budget sums of the accepted band candidates (FP64)
    term = np.where(scores <= lt, 10.0 ** (2.0 * scores.astype(np.float64)), 0.0)
    s2 = np.sqrt(np.add.reduceat(np.append(term, 0.0), off[:-1])) * (np.diff(off) > 0)
    v = np.sort(s2[s2 > 0])
    lo, hi = int(0.4 * v.size), int(0.6 * v.size)
    k = lo + int(np.argmax(np.diff(v[lo:hi])))
    budget = float(0.5 * (v[k] + v[k + 1]))
    T.set_mac(net, 0.3, 1.0, tau, budget)
    try:
        off2, cells2, scores2, fb = T.mac_trace(0.6)
        assert np.array_equal(fb.astype(bool), s2 > budget)
        assert 0 < fb.sum() < fb.size
        assert np.array_equal(off2, off) and np.array_equal(cells2, cells)
        ref, rfb = _replay(R, 0.6, tau, budget, off, cells, scores)
        assert np.array_equal(rfb, fb)
        _lists_equal(T.lists(0.6), ref)
        # forces under these lists against the oracle's FP64 evaluation of them
        acc, pot = T.forces(0.6, 0.01, path="fused_wave")
        ra, rp = R.forces_lists(ref, 0.01)
        err = oracle.rel_err(acc.cpu().numpy().astype(np.float64), ra)
        assert np.median(err) < 1e-5 and err.max() < 1e-4
        perr = np.abs(pot.cpu().numpy() - rp) / np.abs(rp)
        assert np.median(perr) < 1e-5 and perr.max() < 1e-4
        assert T.mac_stats()["fell_back"] == fb.sum()
    finally:
        T.set_mac(None)


@pytest.mark.parametrize("case", ["never_accept", "all_fall_back", "accept_all_band"])
def test_learned_reductions(setup, case):
    pos, m, T, R, P, net, tau = setup
    theta = 0.6
    if case == "never_accept":      # tau_pair = 0: every band cell is opened -> theta_lo walk
        T.set_mac(net, 0.3, 1.0, 0.0, float("inf"))
        ref_theta = 0.3
    elif case == "all_fall_back":   # negative budget: every group walks with theta
        T.set_mac(net, 0.3, 1.0, tau, -1.0)
        ref_theta = theta
    else:                           # everything in the band accepted -> theta_hi walk
        T.set_mac(net, 0.3, 1.0, 1e30, float("inf"))
        ref_theta = 1.0
    try:
        _lists_equal(T.lists(theta), R.lists(ref_theta))
        acc, pot = T.forces(theta, 0.01)
        # the same lists through the theta path give the same bits
        T.set_mac(None)
        a2, p2 = T.forces(ref_theta, 0.01, path="fused_wave")
        assert np.array_equal(acc.cpu().numpy(), a2.cpu().numpy())
        assert np.array_equal(pot.cpu().numpy(), p2.cpu().numpy())
    finally:
        T.set_mac(None)


def test_learned_rejects_other_paths(setup):
    pos, m, T, R, P, net, tau = setup
    T.set_mac(net, 0.3, 1.0, tau, float("inf"))
    try:
        for p in ("two_pass", "fused_block"):
            with pytest.raises(og.OctgravError):
                T.forces(0.6, 0.01, path=p)
        with pytest.raises(og.OctgravError):
            T.set_mac(net, 0.5, 0.4, tau, 1.0)
    finally:
        T.set_mac(None)


def test_learned_frontier_fallback_kernel(setup, monkeypatch):
    # A tiny LDS queue sends every work item through the global-queue kernel;
    # the lists must not change.
    pos, m, T0, R, P, net, tau = setup
    monkeypatch.setenv("OCTGRAV_LDS_QUEUE", "64")
    T = og.Tree(pos, m, 16, 64)
    T.set_mac(net, 0.3, 1.0, tau, float("inf"))
    off, cells, scores, _ = T.mac_trace(0.6)
    ref, _ = _replay(R, 0.6, tau, 1e30, off, cells, scores)
    _lists_equal(T.lists(0.6), ref)


def test_learned_full_size_in_the_bench_configuration():
    """2^20 Plummer sphere with the shipped network at the operating point the
    benchmark measures (band theta* - 0.015 .. theta* + 0.25 around theta* =
    0.5625, tau_pair 3.46e-4, budget 30 tau_pair): the whole call's lists
    replayed by the oracle bit for bit, and the forces of 300 sampled groups
    within the gates of the oracle's FP64 evaluation of those lists."""
    torch = _torch()
    from paper_1005_5384_amd import learned as L
    pos, m = W.make("plummer1m")
    T = og.Tree(pos, m, 16, 64)
    O = oracle.Tree(pos, m, 16, 64)
    tau = 3.46e-4
    T.set_mac(og.Mlp(L.load_params()), 0.5475, 0.8125, tau, 30 * tau)
    off, cells, scores, fb = T.mac_trace(0.5625)
    g = np.repeat(np.arange(off.size - 1, dtype=np.int32), np.diff(off))
    ref, rfb = O.lists_learned(0.5625, 0.5475, 0.8125, oracle.log10_threshold(tau),
                               30 * tau, replay=(g, cells, scores))
    for a, b in zip(T.lists(0.5625), ref):
        assert np.array_equal(a, b)
    assert np.array_equal(fb, rfb)
    acc, pot = T.forces(0.5625, 1e-3)
    torch.cuda.synchronize()
    sel = np.random.default_rng(11).choice(O.n_groups, 300, replace=False).astype(np.int32)
    ar, pr = O.forces_lists(ref, 1e-3, groups=sel)
    k = ~np.isnan(pr)
    ea = oracle.rel_err(acc.double().cpu().numpy()[k], ar[k])
    ep = oracle.rel_err(pot.double().cpu().numpy()[k], pr[k])
    assert np.median(ea) <= 1e-5 and ea.max() <= 1e-4, (np.median(ea), ea.max())
    assert np.median(ep) <= 1e-5 and ep.max() <= 1e-4, (np.median(ep), ep.max())
    T.set_mac(None)
