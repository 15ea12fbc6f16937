"""Pins of the learned-acceptance oracle (CPU): finite-difference gradients,
the closed-form first Adam step, feature invariants, label limits and
convergence, and the walk's reductions to the plain theta walk."""
import numpy as np
import pytest

import oracle
from paper_1005_5384_amd import workloads as W

NP = 5057


def _params(seed, scale=0.3):
    rng = np.random.default_rng(seed)
    P = rng.normal(0, scale, NP)
    return P


def test_param_count():
    assert oracle.mlp_params() == NP == 12 * 64 + 64 + 64 * 64 + 64 + 64 + 1


def test_gradient_matches_finite_differences():
    # FP64 (no BF16 rounding): back-propagation against central differences.
    rng = np.random.default_rng(1)
    P = _params(2)
    x = rng.normal(0, 1, (16, 12)).astype(np.float32)
    t = rng.normal(-4, 1, 16)
    _, g = oracle.mlp_loss_grad(P, x, t, tau=0.9, round_bf16=False)
    h = 1e-6
    idx = np.concatenate([rng.choice(768, 40, replace=False),          # W1
                          768 + rng.choice(64, 10, replace=False),      # b1
                          832 + rng.choice(4096, 60, replace=False),    # W2
                          4928 + rng.choice(64, 10, replace=False),     # b2
                          4992 + rng.choice(64, 10, replace=False),     # w3
                          [5056]])                                      # b3
    for i in idx:
        Pp, Pm = P.copy(), P.copy()
        Pp[i] += h
        Pm[i] -= h
        lp, _ = oracle.mlp_loss_grad(Pp, x, t, round_bf16=False)
        lm, _ = oracle.mlp_loss_grad(Pm, x, t, round_bf16=False)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1e-3, abs(g[i])) + 1e-9, (i, fd, g[i])


def test_forward_bf16_close_to_fp64():
    rng = np.random.default_rng(3)
    P = _params(4, 0.2)
    x = rng.normal(0, 1, (256, 12)).astype(np.float32)
    y64 = oracle.mlp_forward(P, x, round_bf16=False)
    y16 = oracle.mlp_forward(P, x, round_bf16=True)
    assert np.median(np.abs(y16 - y64)) < 0.02 * np.median(np.abs(y64)) + 0.02


def test_adam_first_step_closed_form():
    # From a zero state the bias-corrected first step is -lr g / (|g| + eps).
    rng = np.random.default_rng(5)
    P = rng.normal(size=NP)
    g = rng.normal(size=NP) * 10.0 ** rng.uniform(-6, 0, NP)
    m, v = np.zeros(NP), np.zeros(NP)
    P0 = P.copy()
    oracle.adam_step(P, m, v, g, 1, lr=1e-3)
    np.testing.assert_allclose(P - P0, -1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-10, atol=1e-15)
    # second step with the same gradient: same direction, magnitude from the moments
    P1 = P.copy()
    oracle.adam_step(P, m, v, g, 2, lr=1e-3)
    mh = (0.9 * 0.1 * g + 0.1 * g) / (1 - 0.9 ** 2)
    vh = (0.999 * 0.001 * g * g + 0.001 * g * g) / (1 - 0.999 ** 2)
    np.testing.assert_allclose(P - P1, -1e-3 * mh / (np.sqrt(vh) + 1e-8), rtol=1e-9, atol=1e-15)


@pytest.fixture(scope="module")
def small():
    pos, m = W.plummer(4096, 31)
    T = oracle.Tree(pos, m, 16, 64)
    return pos, m, T


def test_band_is_between_the_two_angles(small):
    pos, m, T = small
    g, c = T.mac_band(0.3, 1.0)
    assert g.size > 0
    f = T.mac_features(g, c)
    # band: 0.3 < l/d <= 1, i.e. 1 <= d/l < 1/0.3 (up to FP32 rounding of d)
    assert np.all(f[:, 0] >= 1 - 1e-6) and np.all(f[:, 0] < 1 / 0.3 + 1e-5)


def test_feature_invariants(small):
    pos, m, T = small
    g, c = T.mac_band(0.3, 1.0)
    f = T.mac_features(g, c)
    e = T.export()
    assert np.all(f[:, 1] <= 1e-7)                          # M_c <= M_tot
    assert np.all(f[:, 2] >= 0)                             # Frobenius norm
    ext = f[:, 4:7]
    assert np.all(ext >= 0) and np.all(ext <= 1 + 1e-6)     # cell extents within the side
    np.testing.assert_allclose(ext.max(1), 1.0, rtol=1e-6)  # the side is the largest extent
    assert np.all(f[:, 11] <= np.sqrt(3) / 2 + 1e-6)        # com inside the box
    depth = e["depth"][c]
    np.testing.assert_allclose(f[:, 10], np.log2(1 + depth) / np.log2(22), rtol=1e-6)
    # group extents: equal for all candidates of one group up to the scaling by l
    l = e["geo"][c, 3].astype(np.float64)
    gb = e["box"][e["groups"][g]]
    np.testing.assert_allclose(2 ** f[:, 7:10] - 1, (gb[:, 3:] - gb[:, :3]) / l[:, None],
                               rtol=1e-5, atol=1e-6)


def test_labels_single_particle_cells_are_exact(small):
    # A one-particle cell's monopole is the pair force itself (Q = 0), so its
    # label vanishes up to FP64 rounding.  (Such cells have side 0 and are
    # never band candidates; the label is defined for any pair.)
    pos, m, T = small
    e = T.export()
    ad, _ = oracle.direct(pos, m, 0.01)
    cells = np.nonzero(e["topo"][:, 3] == 1)[0][:200]
    assert cells.size > 0
    gfirst = e["topo"][e["groups"], 2]
    gl = np.searchsorted(gfirst, e["topo"][cells, 2], side="right") - 1  # group holding the cell
    g = (gl + T.n_groups // 2) % T.n_groups  # some other group
    lab = T.mac_labels(ad, 0.01, g, cells)
    assert np.all(lab < 1e-12)


def test_label_dumbbell_closed_form():
    # Masses m at (+-a, 0, 0) and a target particle at (d, 0, 0): the target's
    # exact acceleration is m/(d-a)^2 + m/(d+a)^2 toward the dumbbell; its
    # monopole + quadrupole (Q = m a^2 diag(4, -2, -2)) gives 2m/d^2 + 6 m a^2/d^4.
    # The label is their relative difference, O((a/d)^4) as the octupole
    # vanishes by symmetry.
    a, mm = 0.5, 0.25
    labs, ds = [], np.array([4.0, 8.0, 16.0, 32.0])
    for d in ds:
        pos = np.array([[-a, 0, 0], [a, 0, 0], [d, 0, 0]], np.float32)
        m = np.array([mm, mm, 1.0], np.float32)
        T = oracle.Tree(pos, m, 2, 1)
        e = T.export()
        cell = int(np.nonzero((e["topo"][:, 3] == 2) & (e["topo"][:, 1] == 0))[0][0])
        gi = int(np.nonzero(e["topo"][e["groups"], 3] == 1)[0][-1])  # the target's group
        assert e["order"][e["topo"][e["groups"][gi], 2]] == 2
        ad, _ = oracle.direct(pos, m, 1e-7)
        lab = T.mac_labels(ad, 1e-7, [gi], [cell])[0]
        exact = mm / (d - a) ** 2 + mm / (d + a) ** 2
        quad = 2 * mm / d ** 2 + 6 * mm * a * a / d ** 4
        np.testing.assert_allclose(lab, abs(quad - exact) / exact, rtol=1e-6)
        labs.append(lab)
    slope = np.polyfit(np.log(ds), np.log(labs), 1)[0]
    assert -4.3 < slope < -3.7, slope


def test_learned_walk_reductions(small):
    pos, m, T = small
    P = _params(7)
    # tau_pair -> 0: the network never accepts, so every band cell is opened:
    # the lists of the plain walk at theta_lo.
    lists, fb = T.lists_learned(0.5, 0.3, 1.0, -100.0, 1e30, params=P)
    for a, b in zip(lists, T.lists(0.3)):
        assert np.array_equal(a, b)
    assert not fb.any()
    # negative budget: every group falls back to the plain walk at theta.
    lists, fb = T.lists_learned(0.5, 0.3, 1.0, 10.0, -1.0, params=P)
    for a, b in zip(lists, T.lists(0.5)):
        assert np.array_equal(a, b)
    assert fb.all()
    # tau_pair -> infinity, no budget: every band cell accepted = plain walk at theta_hi
    lists, fb = T.lists_learned(0.5, 0.3, 1.0, 100.0, 1e30, params=P)
    for a, b in zip(lists, T.lists(1.0)):
        assert np.array_equal(a, b)


def test_learned_walk_replay_matches_network(small):
    pos, m, T = small
    rng = np.random.default_rng(8)
    P = _params(8, 0.1)
    g, c = T.mac_band(0.3, 1.0)
    s = oracle.mlp_forward(P, T.mac_features(g, c)).astype(np.float32)
    thr = float(np.median(s))
    a, fa = T.lists_learned(0.6, 0.3, 1.0, thr, 1e30, params=P)
    b, fb = T.lists_learned(0.6, 0.3, 1.0, thr, 1e30, replay=(g, c, s))
    for x, y in zip(a, b):
        assert np.array_equal(x, y)
    # the learned lists still cover every particle exactly once per group
    e = T.export()
    c_off, c_ids, l_off, l_ids = a
    for gi in rng.choice(T.n_groups, 20, replace=False):
        cover = np.zeros(pos.shape[0], np.int64)
        for cc in np.concatenate([c_ids[c_off[gi]:c_off[gi + 1]], l_ids[l_off[gi]:l_off[gi + 1]]]):
            cover[e["topo"][cc, 2]:e["topo"][cc, 2] + e["topo"][cc, 3]] += 1
        assert np.all(cover == 1)


def test_log10_threshold_is_the_fp64_logarithm_rounded_once():
    # exact decades and a power of two: log10 known in closed form
    assert oracle.log10_threshold(1.0) == 0.0
    assert oracle.log10_threshold(1e-3) == -3.0  # FP32(1e-3) is within 1e-10 relative of 1e-3
    assert oracle.log10_threshold(2.0 ** -10) == float(np.float32(-10 * 0.30102999566398120))
    # the tie that separates it from an FP32 log10: 3.7855e-4 rounds to -3.4218767
    assert oracle.log10_threshold(3.7855e-4) == float(np.float32(-3.4218767))


def test_features_closed_form_two_pairs():
    # Four particles with n_leaf = n_group = 2: the root's octant-0 child holds
    # the pair A (the group), its octant-7 child the pair B (the candidate
    # cell), both leaves and groups.  Every feature of (A, B) follows from the
    # geometry by hand:
    #   B = masses 1 at (5.5, 5.5, 6) and 3 at (6.5, 6.5, 6): tight box side
    #   l = 1 (extents 1, 1, 0), boundary centre (6, 6, 6), centre of mass
    #   (6.25, 6.25, 6); a pair's traceless quadrupole is
    #   mu (3 D D^T - |D|^2 I) with mu = m1 m2 / (m1 + m2) = 3/4 and D = (1, 1, 0),
    #   so |Q|_F = mu |D|^2 sqrt(6) = 1.5 sqrt(6) (off-diagonal Q_xy = 9/4 carries
    #   most of it).
    #   A = masses 2 at (0, 0, 0) and (1, 0.5, 0.25): box extents (1, 0.5, 0.25),
    #   half-diagonal r_g = sqrt(1.3125) / 2; M_tot = 8, M_B = 4.
    pos = np.array([[0, 0, 0], [1, 0.5, 0.25], [5.5, 5.5, 6], [6.5, 6.5, 6]], np.float32)
    m = np.array([2, 2, 1, 3], np.float32)
    T = oracle.Tree(pos, m, 2, 2)
    e = T.export()
    assert T.n_groups == 2 and list(e["groups"]) == [1, 2]
    assert e["topo"][2, 1] == 0 and list(e["topo"][2, 2:]) == [2, 2]  # B: a leaf of 2
    f = T.mac_features(np.array([0], np.int32), np.array([2], np.int32))[0].astype(np.float64)
    l = 1.0
    gext = np.array([1.0, 0.5, 0.25])
    d = np.sqrt((6 - 1.0) ** 2 + (6 - 0.5) ** 2 + (6 - 0.25) ** 2)  # centre to the box
    ref = np.array([
        d / l,
        np.log10(4 / 8) / 3,
        1.5 * np.sqrt(6) / (4 * l * l),
        np.log2(1 + 0.5 * np.sqrt(1.3125) / l),
        1.0, 1.0, 0.0,
        *np.log2(1 + gext / l),
        np.log2(1 + 1) / np.log2(22),                      # B sits at depth 1
        np.sqrt(2 * 0.25 ** 2) / l,                        # |com - boundary centre| / l
    ])
    np.testing.assert_allclose(f, ref, rtol=2e-6, atol=1e-7)


def test_forward_single_paths_closed_form():
    # Two paths through an otherwise zero network, weights and inputs exact in
    # BF16: y = w3[a] relu(W2[a, b] h_b + W2[a, c] h_c + b2[a]) + b3 with
    # h_b = relu(W1[b, k] x_k + b1[b]), h_c = relu(W1[c, j] x_j + b1[c]).  A
    # transposed W1 or W2 reads other (zero) entries and gives b3 + w3 relu(b2).
    a, b, c, k, j = 5, 17, 40, 3, 11
    P = np.zeros(NP)
    P[b * 12 + k] = 1.5                # W1[b, k]
    P[c * 12 + j] = -0.75              # W1[c, j]
    P[768 + b] = 0.25                  # b1[b]
    P[768 + c] = 1.0                   # b1[c]
    P[832 + a * 64 + b] = -2.0         # W2[a, b]
    P[832 + a * 64 + c] = 0.5          # W2[a, c]
    P[4928 + a] = 4.0                  # b2[a]
    P[4992 + a] = 0.5                  # w3[a]
    P[5056] = 0.125                    # b3
    x = np.zeros((64, 12), np.float32)
    i = np.arange(64)
    x[:, k] = (i % 16) / 4 - 2         # multiples of 1/4: every value below has at most
    x[:, j] = 1 - (i // 4) / 4         # 8 significant bits, so BF16 rounding is exact
    hb = np.maximum(1.5 * x[:, k] + 0.25, 0)
    hc = np.maximum(-0.75 * x[:, j] + 1.0, 0)
    ref = 0.5 * np.maximum(-2.0 * hb + 0.5 * hc + 4.0, 0) + 0.125
    for rnd in (False, True):
        y = oracle.mlp_forward(P, x, round_bf16=rnd)
        np.testing.assert_allclose(y, ref, rtol=0, atol=1e-12)
    assert np.ptp(ref) > 1.0
