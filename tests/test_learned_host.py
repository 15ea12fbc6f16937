"""Host logic of the learned criterion's driver (CPU): the bisection used
for the equal-error comparison, and the parameter file."""
import numpy as np

from paper_1005_5384_amd import learned as L


def test_bisect_increasing_hits_target_from_below():
    f = lambda x: x ** 3
    x, v = L.bisect(f, 0.0, 2.0, 1.0, increasing=True, iters=30, rtol=1e-3)
    assert v <= 1.0 and abs(v - 1.0) <= 1e-3


def test_bisect_decreasing():
    f = lambda x: 1.0 / x
    x, v = L.bisect(f, 0.5, 8.0, 0.25, increasing=False, iters=30, rtol=1e-3)
    assert v <= 0.25 and abs(x - 4.0) < 0.01


def test_bisect_unreachable_target_returns_safe_end():
    x, v = L.bisect(lambda x: x + 10.0, 0.0, 1.0, 1.0, increasing=True, iters=5)
    assert x == 0.0 and v == 10.0


def test_init_params_shape_and_bias():
    P = L.init_params(0)
    assert P.dtype == np.float32 and P.shape == (5057,)
    assert P[5056] == -4.0 and np.all(P[768:832] == 0)


def _ckpt(seed=1):
    rng = np.random.default_rng(seed)
    p = rng.normal(size=5057).astype(np.float32)
    m1 = rng.normal(size=5057).astype(np.float32)
    m2 = np.abs(rng.normal(size=5057)).astype(np.float32)
    gen = rng.integers(0, 256, 5056).astype(np.uint8)
    return L.pack_checkpoint(p, m1, m2, 120, 3, gen, [30, 4096, 1e-3, 1e-4, 0.9, 0])


def test_checkpoint_round_trip(tmp_path):
    a = _ckpt()
    path = str(tmp_path / "ck.npz")
    L.save_checkpoint(path, a)
    b = L.load_checkpoint(path)
    for k in L.CKPT_KEYS:
        assert np.array_equal(a[k], b[k]) and a[k].dtype == b[k].dtype, k
    assert int(b["step"]) == 120 and int(b["epoch"]) == 3


def test_checkpoint_rejects_corruption_version_and_shape(tmp_path):
    import pytest
    a = _ckpt()
    path = str(tmp_path / "ck.npz")
    # one flipped bit in a moment
    bad = dict(a)
    m2 = a["mom2"].copy()
    m2.view(np.uint32)[17] ^= 1
    bad["mom2"] = m2
    L.save_checkpoint(path, bad)
    with pytest.raises(ValueError, match="checksum"):
        L.load_checkpoint(path)
    # another format version (checksum recomputed, so only the version differs)
    other = dict(a)
    other["version"] = np.int64(L.CKPT_VERSION + 1)
    other["sha256"] = L._ckpt_digest(other)
    L.save_checkpoint(path, other)
    with pytest.raises(ValueError, match="version"):
        L.load_checkpoint(path)
    # a missing array
    np.savez(path, **{k: v for k, v in a.items() if k != "mom1"})
    with pytest.raises(ValueError, match="missing"):
        L.load_checkpoint(path)
    with pytest.raises(ValueError):
        L.pack_checkpoint(a["params"][:100], a["mom1"], a["mom2"], 1, 1, a["gen_state"],
                          a["settings"])
