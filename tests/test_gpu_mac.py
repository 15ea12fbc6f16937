"""GPU parity of the learned acceptance criterion's pieces (through the C
ABI) against the FP64 oracle: direct summation, band candidates, features
and labels."""
import numpy as np
import pytest

import oracle
from paper_1005_5384_amd import octgrav as og
from paper_1005_5384_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def plummer():
    import torch
    assert torch.cuda.is_available()
    pos, m = W.plummer(8192, 41)
    return pos, m, og.Tree(pos, m, 16, 64), oracle.Tree(pos, m, 16, 64)


@pytest.mark.parametrize("sel", [None, "sample"])
def test_direct_matches_oracle(plummer, sel):
    pos, m, T, _ = plummer
    eps = 0.01
    tg = None if sel is None else W.sample_indices(pos.shape[0], 1000, 5)
    acc, pot = T.direct(eps, tg)
    ra, rp = oracle.direct(pos, m, eps, tg)
    err = oracle.rel_err(acc.cpu().numpy().astype(np.float64), ra)
    assert np.median(err) < 1e-6 and err.max() < 1e-5, (np.median(err), err.max())
    perr = np.abs(pot.cpu().numpy() - rp) / np.abs(rp)
    assert perr.max() < 1e-5


def test_direct_empty_targets(plummer):
    _, _, T, _ = plummer
    acc, pot = T.direct(0.01, [])
    assert acc.shape == (0, 3)


def _key(g, c):
    return np.asarray(g, np.int64) << 32 | np.asarray(c, np.int64)


@pytest.mark.parametrize("stride", [1, 7])
def test_band_features_labels_match_oracle(plummer, stride):
    pos, m, T, R = plummer
    eps = 0.01
    ad, _ = T.direct(eps)
    feat, lab, gid, cid = T.mac_collect(eps, ad, 0.3, 1.0, stride=stride)
    feat, lab = feat.cpu().numpy(), lab.cpu().numpy()
    gid, cid = gid.cpu().numpy(), cid.cpu().numpy()
    groups = np.arange(0, R.n_groups, stride)
    rg, rc = R.mac_band(0.3, 1.0, groups=groups)
    # the same candidate set, in the same order (groups ascending, each
    # group's candidates in walk order)
    assert gid.size == rg.size > 0
    assert np.array_equal(gid, rg) and np.array_equal(cid, rc)
    rf = R.mac_features(rg, rc)
    # hardware reciprocal, square root and log2 on the GPU (about 1 ulp each)
    np.testing.assert_allclose(feat, rf, rtol=1e-5, atol=1e-6)
    rad, _ = oracle.direct(pos, m, eps)
    rl = R.mac_labels(rad, eps, rg, rc)
    big = rl >= 1e-6
    assert big.sum() > 0.5 * rl.size
    assert np.all(np.abs(lab - rl) <= 0.02 * rl + 2e-7), np.max(np.abs(lab - rl) / (rl + 1e-7))
    # the log-labels the network is trained on agree within 0.05 dex
    assert np.all(np.abs(np.log10(lab[big]) - np.log10(rl[big])) < 0.05)


def test_collect_capacity_truncates_at_group_boundary(plummer):
    pos, m, T, R = plummer
    ad, _ = T.direct(0.01)
    f_all, _, g_all, _ = T.mac_collect(0.01, ad)
    cap = int(f_all.shape[0] // 3)
    f, _, g, _ = T.mac_collect(0.01, ad, cap=cap)
    g, g_all = g.cpu().numpy(), g_all.cpu().numpy()
    assert 0 < g.size <= cap
    # only whole groups are kept
    last = g[-1]
    assert np.sum(g_all == last) == np.sum(g == last)
    assert np.array_equal(g, g_all[:g.size])


def test_direct_rejects_bad_targets(plummer):
    _, _, T, _ = plummer
    with pytest.raises(og.OctgravError):
        T.direct(0.01, [0, T.n])
