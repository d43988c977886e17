"""Pin of the whole oracle scheme (score, damping, Euler-Maruyama step, noise) against the
closed-form mean/variance recursion of a Gaussian prior with a linear observation."""
import numpy as np
import pytest
from scipy.stats import norm

from oracle import ensf
from oracle import linear_gaussian as lg


def quantile_members(mu, n):
    """n members of N(mu, 1) placed at the normal quantiles (j + 1/2)/n: a deterministic
    sample whose empirical law differs from the Gaussian by O(1/n) in smooth functionals,
    so the finite-ensemble error of the Monte-Carlo score stays far below the particles'
    sampling error at n = 2048 (a random sample would add an O(1/sqrt(n)) offset)."""
    return (mu + norm.ppf((np.arange(n) + 0.5) / n))[:, None]


@pytest.mark.parametrize("sigma_o,y,K,seed", [(1.0, 1.0, 100, 7), (0.5, -0.5, 200, 8)])
def test_particles_follow_discrete_recursion(sigma_o, y, K, seed):
    N, P = 2048, 1024
    X = quantile_members(0.3, N)
    Z = ensf.analysis(X, np.array([0]), np.array([y]), sigma_o, K, seed=seed,
                      obs_op="linear", n_particles=P, chunk=256)
    mh, s2h = X[:, 0].mean(), X[:, 0].var(ddof=1)
    m, v = lg.em_recursion(mh, s2h, y / sigma_o ** 2, 1.0 / sigma_o ** 2, K)
    # particle sampling error only: 4 standard errors of the mean, chi-square band of the
    # variance (the particles are independent draws)
    assert abs(Z[:, 0].mean() - m) < 4 * np.sqrt(v / P)
    assert abs(Z[:, 0].var(ddof=1) / v - 1.0) < 4 * np.sqrt(2.0 / (P - 1))


def test_particles_resample_prior_without_observations():
    N, P, K = 2048, 1024, 50
    X = quantile_members(-0.4, N)
    Z = ensf.analysis(X, np.zeros(0, dtype=np.int64), np.zeros(0), 1.0, K, seed=13,
                      obs_op="linear", n_particles=P, chunk=256)
    m, v = lg.em_recursion(X[:, 0].mean(), X[:, 0].var(ddof=1), 0.0, 0.0, K)
    assert abs(Z[:, 0].mean() - m) < 4 * np.sqrt(v / P)
    assert abs(Z[:, 0].var(ddof=1) / v - 1.0) < 4 * np.sqrt(2.0 / (P - 1))


def test_recursion_reduces_to_prior_without_observations():
    # no likelihood: the exact-score scheme must return (approximately, O(dt)) the prior
    m, v = lg.em_recursion(0.4, 2.0, 0.0, 0.0, 4000)
    assert abs(m - 0.4) < 5e-3 and abs(v - 2.0) < 5e-3


def test_kalman_gap_is_bounded_and_reported():
    # the damped score h(t) = 1 - t is not the Bayes posterior score: report the gap
    for s2o in (0.25, 1.0, 4.0):
        m, v = lg.em_recursion(0.0, 1.0, 1.0 / s2o, 1.0 / s2o, 1000)
        km, kv = lg.kalman(0.0, 1.0, 1.0, s2o)
        assert abs(m - km) < 0.3 * np.sqrt(kv)
        assert 0.5 * kv < v < 1.5 * kv


def test_recursion_is_unstable_when_dt_exceeds_obs_variance():
    # explicit EM needs dt of order sigma_o^2 or smaller (stiff likelihood term near t = 0)
    m100, _ = lg.em_recursion(0.0, 1.0, 1.0 / 0.0025, 1.0 / 0.0025, 100)
    m1000, _ = lg.em_recursion(0.0, 1.0, 1.0 / 0.0025, 1.0 / 0.0025, 1000)
    assert abs(m100) > 1e3
    assert abs(m1000 - 1.0) < 0.05
