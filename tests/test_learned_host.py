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
