"""GPU parity of the HIP path (through the C ABI) against the FP64 oracle.

Lists must match bit-exactly; accelerations and potentials must lie within
a 1e-5 median and 1e-4 max relative error of the oracle's same-tree FP64
evaluation.  Particles whose reference acceleration is below 1e-6 of the
median are reported apart and kept out of the max gate."""
import os

import numpy as np
import pytest

import oracle
from paper_1005_5384_amd import octgrav as og
from paper_1005_5384_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL_MED, TOL_MAX = 1e-5, 1e-4


def _torch():
    import torch
    assert torch.cuda.is_available()
    return torch


PATHS = ("two_pass", "fused_block", "fused_wave")


def _lists_all_paths(T, theta, ref):
    _lists_equal(T.lists(theta), ref)
    for p in PATHS:
        _lists_equal(T.lists(theta, path=p), ref)


def _lists_equal(gpu, orc):
    names = ("c_off", "c_ids", "l_off", "l_ids")
    for name, a, b in zip(names, gpu, orc):
        assert a.shape == b.shape, name
        assert np.array_equal(a, b), name


def _gate(a, p, a_ref, p_ref, what=""):
    na = np.linalg.norm(a_ref, axis=1)
    keep = na >= 1e-6 * np.median(na)
    ea = oracle.rel_err(a[keep], a_ref[keep])
    ep = oracle.rel_err(p, p_ref)
    msg = f"{what} acc med {np.median(ea):.3g} max {ea.max():.3g} pot med {np.median(ep):.3g} max {ep.max():.3g}"
    print(msg)
    assert np.median(ea) <= TOL_MED and ea.max() <= TOL_MAX, msg
    assert np.median(ep) <= TOL_MED and ep.max() <= TOL_MAX, msg
    return np.median(ea), ea.max()


def _gpu_forces(T, theta, eps, **kw):
    torch = _torch()
    a, p = T.forces(theta, eps, **kw)
    torch.cuda.synchronize()
    return a.double().cpu().numpy(), p.double().cpu().numpy()


# ------------------------------------------------------------------ lists
@pytest.mark.parametrize("n,n_leaf,n_group,seed", [(10, 16, 64, 1), (600, 4, 16, 21),
                                                   (3000, 1, 1, 5), (2500, 8, 32, 7),
                                                   (5000, 64, 64, 8)])
@pytest.mark.parametrize("theta", [0.0, 0.3, 0.6, 1.0])
def test_lists_small_variety(n, n_leaf, n_group, seed, theta):
    pos, m = W.plummer(n, seed)
    T = og.Tree(pos, m, n_leaf, n_group)
    ref = oracle.Tree(pos, m, n_leaf, n_group).lists(theta)
    _lists_all_paths(T, theta, ref)


@pytest.fixture(scope="module")
def c1():
    w = W.WORKLOADS["plummer16k"]
    pos, m = W.make("plummer16k")
    return pos, m, w, og.Tree(pos, m, w["n_leaf"], 64), oracle.Tree(pos, m, w["n_leaf"], 64)


@pytest.mark.parametrize("theta", [0.0, 0.3, 0.5, 0.75, 1.0])
def test_lists_c1(c1, theta):
    pos, m, w, T, O = c1
    _lists_all_paths(T, theta, O.lists(theta))


@pytest.fixture(scope="module")
def c2():
    w = W.WORKLOADS["plummer1m"]
    pos, m = W.make("plummer1m")
    return pos, m, w, og.Tree(pos, m, w["n_leaf"], 64), oracle.Tree(pos, m, w["n_leaf"], 64)


@pytest.mark.parametrize("theta", [0.3, 0.5, 0.75])
def test_lists_c2_full(c2, theta):
    pos, m, w, T, O = c2
    _lists_all_paths(T, theta, O.lists(theta))


def test_lists_clumps_full():
    w = W.WORKLOADS["clumps4m"]
    pos, m = W.make("clumps4m")
    T = og.Tree(pos, m, w["n_leaf"], 64)
    O = oracle.Tree(pos, m, w["n_leaf"], 64)
    _lists_equal(T.lists(0.5), O.lists(0.5))
    sel = np.random.default_rng(3).choice(O.n_groups, 200, replace=False)
    a, p = _gpu_forces(T, 0.5, w["eps"])
    ar, pr = O.forces(0.5, w["eps"], groups=sel)
    k = ~np.isnan(pr)
    _gate(a[k], p[k], ar[k], pr[k], "clumps4m sampled")


def test_lists_select_equals_slices(c1):
    # The selected-group export (for trees whose full lists do not fit on the
    # host) gives the full lists' slices, in the selection's order, repeats
    # and an empty selection included, on every path and against the oracle's
    # own selection.
    pos, m, w, T, O = c1
    ng = O.n_groups
    sel = np.array([ng - 1, 0, 5, 5, ng // 2, 1], np.int32)
    full = O.lists(0.5)
    ref = O.lists(0.5, groups=sel)
    c_off, c_ids, l_off, l_ids = full
    for k, g in enumerate(sel):
        assert np.array_equal(ref[1][ref[0][k]:ref[0][k + 1]], c_ids[c_off[g]:c_off[g + 1]])
        assert np.array_equal(ref[3][ref[2][k]:ref[2][k + 1]], l_ids[l_off[g]:l_off[g + 1]])
    for p_ in (None,) + PATHS:
        _lists_equal(T.lists(0.5, path=p_, groups=sel), ref)
    empty = T.lists(0.5, groups=np.zeros(0, np.int32))
    assert empty[0].tolist() == [0] and empty[1].size == 0 and empty[3].size == 0
    for bad in ([-1], [ng]):
        with pytest.raises(og.OctgravError, match="outside"):
            T.lists(0.5, groups=np.array(bad, np.int32))


def test_lists_via_fallback_walk(c1):
    # A 64-entry LDS frontier overflows for almost every group, so the lists
    # come from the global-memory fallback walk; they must not change.
    pos, m, w, _, O = c1
    os.environ["OCTGRAV_LDS_QUEUE"] = "64"
    try:
        T = og.Tree(pos, m, w["n_leaf"], 64)
    finally:
        del os.environ["OCTGRAV_LDS_QUEUE"]
    for theta in (0.3, 0.75):
        _lists_all_paths(T, theta, O.lists(theta))
    ar, pr = O.forces(0.5, w["eps"])
    for p_ in PATHS:
        a, p = _gpu_forces(T, 0.5, w["eps"], path=p_)
        _gate(a, p, ar, pr, f"fallback walk path={p_}")


# ------------------------------------------------------------------ forces
@pytest.mark.parametrize("path", PATHS)
@pytest.mark.parametrize("theta", [0.3, 0.5, 0.75])
def test_forces_c1(c1, theta, path):
    pos, m, w, T, O = c1
    a, p = _gpu_forces(T, theta, w["eps"], path=path)
    ar, pr = O.forces(theta, w["eps"])
    _gate(a, p, ar, pr, f"c1 theta={theta} path={path}")


@pytest.mark.parametrize("path", PATHS)
@pytest.mark.parametrize("theta", [0.3, 0.5, 0.75])
def test_forces_c2_sampled(c2, theta, path):
    pos, m, w, T, O = c2
    sel = np.random.default_rng(int(theta * 100)).choice(O.n_groups, 400, replace=False)
    a, p = _gpu_forces(T, theta, w["eps"], path=path)
    ar, pr = O.forces(theta, w["eps"], groups=sel)
    k = ~np.isnan(pr)
    _gate(a[k], p[k], ar[k], pr[k], f"c2 theta={theta} path={path}")
    # interaction totals reported by the library equal the oracle's counts
    cnt = O.counts(theta)
    gs = O.export()["topo"][O.export()["groups"], 3]
    lc = T.last_counts()
    assert lc["n_c"] == cnt[:, 0].sum() and lc["n_l"] == cnt[:, 1].sum()
    assert lc["n_pc"] == (cnt[:, 0] * gs).sum() and lc["n_pp"] == (cnt[:, 2] * gs).sum()
    # and so do the per-group list lengths, group by group
    assert np.array_equal(T.group_counts()[:, :3], cnt)


def test_plain_vs_compensated(c2):
    pos, m, w, T, O = c2
    sel = np.random.default_rng(7).choice(O.n_groups, 400, replace=False)
    ar, pr = O.forces(0.5, w["eps"], groups=sel)
    k = ~np.isnan(pr)
    ak, pk = _gpu_forces(T, 0.5, w["eps"])
    ap, pp = _gpu_forces(T, 0.5, w["eps"], plain=True)
    ek = oracle.rel_err(ak[k], ar[k])
    ep = oracle.rel_err(ap[k], ar[k])
    print(f"compensated med {np.median(ek):.3g} max {ek.max():.3g}; "
          f"plain med {np.median(ep):.3g} max {ep.max():.3g}")
    _gate(ak[k], pk[k], ar[k], pr[k], "compensated")
    assert np.median(ek) <= np.median(ep) * 1.05


def test_theta_zero_equals_direct():
    pos, m = W.plummer(4096, 9)
    T = og.Tree(pos, m, 8, 32)
    a, p = _gpu_forces(T, 0.0, 0.01)
    ad, pd = oracle.direct(pos, m, 0.01)
    _gate(a, p, ad, pd, "theta=0 vs direct")


def test_diagnostics_fp64(c1):
    pos, m, w, T, O = c1
    a, p = _gpu_forces(T, 0.5, w["eps"])
    mom, wp = T.diagnostics()
    mom_ref, w_ref = oracle.diagnostics(m, a, p)
    scale = np.sum(m.astype(np.float64) * np.linalg.norm(a, axis=1))
    assert np.all(np.abs(mom - mom_ref) <= 1e-12 * scale)
    assert abs(wp - w_ref) <= 1e-12 * abs(w_ref)
    # the tree force does not conserve momentum exactly, but nearly
    assert np.all(np.abs(mom) <= 1e-3 * scale)


@pytest.mark.parametrize("path", PATHS)
def test_repeatable_bitwise(c1, path):
    pos, m, w, T, O = c1
    a1, p1 = _gpu_forces(T, 0.5, w["eps"], path=path)
    a2, p2 = _gpu_forces(T, 0.5, w["eps"], path=path)
    assert np.array_equal(a1, a2) and np.array_equal(p1, p2)


def test_paths_agree(c2):
    # Same lists, different tile interleaving: results agree to rounding.
    pos, m, w, T, O = c2
    ref, _ = _gpu_forces(T, 0.5, w["eps"], path="two_pass")
    for p_ in ("fused_block", "fused_wave"):
        a, _ = _gpu_forces(T, 0.5, w["eps"], path=p_)
        e = oracle.rel_err(a, ref)
        assert np.median(e) < 1e-6 and e.max() < 1e-4


def test_capacity_regrowth(c1):
    # Small lists first, then larger ones on the same handle: the list
    # buffers are regrown inside the call and the result is still exact.
    pos, m, w, _, O = c1
    T = og.Tree(pos, m, w["n_leaf"], 64)
    _gpu_forces(T, 1.0, w["eps"], two_pass=True)
    a, p = _gpu_forces(T, 0.3, w["eps"], two_pass=True)
    ar, pr = O.forces(0.3, w["eps"])
    _gate(a, p, ar, pr, "regrowth")


def test_pot_optional_and_stream(c1):
    torch = _torch()
    pos, m, w, T, O = c1
    a0, p0 = _gpu_forces(T, 0.5, w["eps"])
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        acc, pot = T.forces(0.5, w["eps"], with_pot=False)
    s.synchronize()
    assert pot is None
    assert np.array_equal(acc.double().cpu().numpy(), a0)


# ------------------------------------------------------------------ edge cases
def test_single_particle():
    T = og.Tree(np.array([[1.0, 2.0, 3.0]], np.float32), np.ones(1, np.float32))
    a, p = _gpu_forces(T, 0.5, 0.1)
    assert np.all(a == 0) and np.all(p == 0)


def test_two_bodies():
    pos = np.array([[0.1, -0.2, 0.3], [0.6, 0.4, -0.2]], np.float32)
    m = np.array([0.25, 0.75], np.float32)
    T = og.Tree(pos, m, 1, 1)
    a, p = _gpu_forces(T, 0.5, 0.05)
    ad, pd = oracle.direct(pos, m, 0.05)
    _gate(a, p, ad, pd, "two bodies")


def test_coincident_stacks_and_big_groups():
    # depth-21 leaves holding 150 and 100 coincident particles: groups larger
    # than 64 targets are evaluated in chunks
    rng = np.random.default_rng(1)
    pos = np.concatenate([np.zeros((150, 3)), np.ones((100, 3)) * [0.5, 0.25, -0.5],
                          rng.normal(size=(500, 3))]).astype(np.float32)
    m = rng.uniform(0.5, 1.5, 750).astype(np.float32) / 750
    T = og.Tree(pos, m, 8, 64)
    assert T.stats["n_work"] > T.stats["n_groups"]
    O = oracle.Tree(pos, m, 8, 64)
    for theta in (0.0, 0.5, 1.0):
        _lists_all_paths(T, theta, O.lists(theta))
        ar, pr = O.forces(theta, 0.02)
        for p_ in PATHS:
            a, p = _gpu_forces(T, theta, 0.02, path=p_)
            _gate(a, p, ar, pr, f"coincident theta={theta} path={p_}")


def test_ragged_sizes_match_oracle():
    for n, seed in ((65, 2), (1023, 3), (4097, 4)):
        pos, m = W.plummer(n, seed)
        T = og.Tree(pos, m, 16, 64)
        O = oracle.Tree(pos, m, 16, 64)
        a, p = _gpu_forces(T, 0.5, 0.01)
        ar, pr = O.forces(0.5, 0.01)
        _gate(a, p, ar, pr, f"n={n}")


def test_bad_arguments_rejected(c1):
    torch = _torch()
    pos, m, w, T, O = c1
    acc = torch.empty((T.n, 3), dtype=torch.float32, device="cuda")
    for theta, eps in ((1.5, 0.01), (-0.1, 0.01), (float("nan"), 0.01), (0.5, 0.0), (0.5, -1.0)):
        with pytest.raises(og.OctgravError) as ei:
            T.forces(theta, eps, acc=acc)
        assert ei.value.code == og.EINVAL


def test_group_counts_need_a_call():
    pos, m = W.plummer(2048, 5)
    T = og.Tree(pos, m, 16, 64)
    with pytest.raises(og.OctgravError, match="no completed"):
        T.group_counts()
    _gpu_forces(T, 0.6, 0.01)
    gc = T.group_counts()
    assert gc.shape == (T.stats["n_groups"], 4) and (gc[:, 3] == 0).all()
