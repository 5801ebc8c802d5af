"""Pins of the oracle's UpdateMean / UpdateCov.

MPPI (Sec. III-C, Alg. 4): normalised weights against scipy's softmax, their
sum, the lambda -> 0 (argmin) and lambda -> infinity (plain mean) limits,
invariance to a cost offset and to sample order.
Elite (Alg. 1, top K_e after sorting) and naive (Alg. 3, best sample): brute
force with numpy sorting, mean and ddof=0 variance on tiny inputs.
"""
import math

import numpy as np
from scipy.special import softmax


def test_mppi_weights_match_softmax(orc):
    rng = np.random.default_rng(0)
    for lam in (0.3, 1.0, 7.0):
        J = rng.uniform(0, 40, size=300)
        w, beta, Om, flags = orc.mppi_weights(J, lam)
        assert flags == 0 and beta == J.min()
        np.testing.assert_allclose(w, softmax(-J / lam), rtol=1e-12, atol=1e-300)
        assert abs(w.sum() - 1.0) <= J.size * 2.0**-52
        assert abs(Om - np.exp(-(J - J.min()) / lam).sum()) <= 1e-12 * Om


def test_mppi_lambda_to_zero_is_argmin(orc):
    rng = np.random.default_rng(1)
    J = rng.permutation(np.arange(50, dtype=np.float64) * 0.37 + 2.0)
    theta = rng.normal(size=(50, 7))
    w, *_ = orc.mppi_weights(J, 1e-9)
    mean = orc.weighted_mean(w, theta)
    np.testing.assert_array_equal(mean, theta[np.argmin(J)])


def test_mppi_lambda_to_infinity_is_mean(orc):
    rng = np.random.default_rng(2)
    J = rng.uniform(0, 10, size=64)
    theta = rng.normal(size=(64, 5))
    w, *_ = orc.mppi_weights(J, 1e12)
    np.testing.assert_allclose(orc.weighted_mean(w, theta), theta.mean(0), rtol=1e-9, atol=1e-12)


def test_mppi_shift_and_permutation_invariance(orc):
    rng = np.random.default_rng(3)
    J = rng.uniform(0, 20, size=100)
    theta = rng.normal(size=(100, 4))
    w1, *_ = orc.mppi_weights(J, 1.0)
    w2, *_ = orc.mppi_weights(J + 1234.5, 1.0)
    np.testing.assert_allclose(w1, w2, rtol=1e-9)
    perm = rng.permutation(100)
    w3, *_ = orc.mppi_weights(J[perm], 1.0)
    np.testing.assert_allclose(orc.weighted_mean(w3, theta[perm]), orc.weighted_mean(w1, theta),
                               rtol=1e-12, atol=1e-14)


def test_mppi_nonfinite(orc):
    w, beta, Om, flags = orc.mppi_weights(np.full(5, np.inf), 1.0)
    assert flags == 1 and beta == math.inf and np.all(w == 0)
    J = np.array([np.inf, 3.0, np.inf, 4.0])
    w, beta, Om, flags = orc.mppi_weights(J, 1.0)
    assert flags == 0 and w[0] == 0 and w[2] == 0
    np.testing.assert_allclose(w[[1, 3]], softmax([-3.0, -4.0]), rtol=1e-14)


def test_elite_select_brute_force(orc):
    rng = np.random.default_rng(4)
    for n in range(1, 9):
        for _ in range(30):
            J = rng.integers(0, 4, size=n).astype(np.float64)  # many ties
            for ke in range(1, n + 1):
                order = np.lexsort((np.arange(n), J))  # by cost, then index
                np.testing.assert_array_equal(orc.elite_select(J, ke), order[:ke])


def test_elite_moments_match_numpy(orc):
    rng = np.random.default_rng(5)
    theta = rng.normal(size=(8, 6)) * 3
    for ke in range(1, 9):
        idx = rng.permutation(8)[:ke].astype(np.int32)
        mean, var = orc.elite_moments(idx, theta)
        np.testing.assert_allclose(mean, theta[idx].mean(0), rtol=1e-14, atol=1e-15)
        np.testing.assert_allclose(var, theta[idx].var(0, ddof=0), rtol=1e-12, atol=1e-15)


def test_elite_count(orc):
    assert orc.elite_count(16384, 0.1) == 1638
    assert orc.elite_count(5, 0.1) == 1
    assert orc.elite_count(10, 1.0) == 10
    assert orc.elite_count(10, 2.0) == 10
