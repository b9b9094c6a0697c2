"""Pins of the oracle's dynamic-static split and static constraint (Section 4.1,
Eqs. 4-5) against brute force and closed forms."""
import math

import numpy as np

from oracle import hash4d_oracle as O


def brute_force_split(dp, k):
    """Count, for every Gaussian, how many have a strictly larger FP32 squared
    magnitude (NaN ranked above everything); the top floor(k n / 100) by that rank,
    without the ones tied with the first excluded key, are dynamic."""
    key = O.motion_keys(dp).astype(np.int64)
    n = len(key)
    n_d = int(math.floor(k / 100.0 * n))
    dyn = []
    for i in range(n):
        at_least = int(np.sum(key >= key[i]))   # rank from the top, ties counted in
        if at_least <= n_d:
            dyn.append(i)
    return np.array(dyn, dtype=np.int64)


def test_split_matches_brute_force_with_ties_and_nan():
    rng = np.random.default_rng(70)
    dp = rng.standard_normal((300, 3)).astype(np.float32)
    dp[10:20] = dp[5]            # ties
    dp[30] = [np.nan, 0, 0]      # ranks above everything
    dp[40:45] = 0.0              # zero motion
    for k in (0, 1, 3.3, 10, 50, 99, 100):
        idx, _, _ = O.decompose(dp, k)
        assert np.array_equal(idx, brute_force_split(dp, k)), k


def test_split_count_is_exact_for_distinct_magnitudes():
    rng = np.random.default_rng(71)
    dp = rng.standard_normal((1000, 3)).astype(np.float32)
    for k in (5, 12.5, 37):
        idx, _, _ = O.decompose(dp, k)
        assert len(idx) == int(math.floor(k / 100 * 1000))
        mags = np.linalg.norm(dp.astype(np.float64), axis=1)
        assert mags[idx].min() > np.delete(mags, idx).max()


def test_static_constraint_value_and_gradient():
    rng = np.random.default_rng(72)
    dp = rng.standard_normal((50, 3)).astype(np.float32)
    dp[7] = 0.0
    idx, loss, grad = O.decompose(dp, 20, lam_s=0.3)
    static = np.setdiff1d(np.arange(50), idx)
    d = dp.astype(np.float64)
    assert math.isclose(loss, 0.3 / len(static) * sum(math.sqrt(float(x @ x)) for x in d[static]), rel_tol=1e-14)
    assert not grad[idx].any() and not grad[7].any()
    # central differences of the loss with the split held fixed
    for i in static[:10]:
        if i == 7:
            continue
        for c in range(3):
            e = np.zeros(3)
            e[c] = 1e-6
            f = lambda v: 0.3 / len(static) * np.linalg.norm(v)
            fd = (f(d[i] + e) - f(d[i] - e)) / 2e-6
            assert abs(fd - grad[i, c]) < 1e-8


def test_linear_motion():
    p = np.array([[0.1, 0.2, 0.3]])
    dp = np.array([[1.0, -2.0, 0.5]])
    assert np.allclose(O.linear_motion(p, np.array([0.5]), dp), [[0.6, -0.8, 0.55]], rtol=0, atol=1e-15)
