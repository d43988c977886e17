"""Pins of the FP64 EnSF oracle against what the paper and the mathematics fix
(brute force, invariants, closed forms, finite differences)."""
import numpy as np
import pytest

from oracle import ensf


def _rand(seed, *shape, scale=1.0):
    return scale * np.random.default_rng(seed).standard_normal(shape)


@pytest.mark.parametrize("t", [1.0, 0.5, 0.1, 0.02])
def test_gram_form_matches_bruteforce(t):
    # distances small enough that exp(-D / 2 beta^2) does not underflow in the brute force
    Z = _rand(1, 3, 5, scale=0.3)
    X = _rand(2, 4, 5, scale=0.3)
    S, W = ensf.prior_score(Z, X, t, return_weights=True)
    Sb, Wb = ensf.prior_score_bruteforce(Z, X, t)
    np.testing.assert_allclose(W, Wb, rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(S, Sb, rtol=1e-11, atol=1e-12)


def test_weights_sum_to_one_even_when_degenerate():
    Z = _rand(3, 16, 4096)
    X = _rand(4, 20, 4096)
    for t in (1.0, 0.5, 0.01):
        W = ensf.prior_weights(Z, X, t)
        assert np.all(W >= 0)
        np.testing.assert_allclose(W.sum(axis=1), 1.0, atol=1e-12)


@pytest.mark.parametrize("t", [1.0, 0.3, 0.0025])
def test_single_member_gives_gaussian_score(t):
    # eq. 12: with one member the score is that of N(alpha x, beta^2 I)
    Z = _rand(5, 4, 33)
    X = _rand(6, 1, 33)
    s = ensf.schedule(t)
    np.testing.assert_allclose(ensf.prior_score(Z, X, t),
                               -(Z - s["alpha"] * X) / s["beta2"], rtol=1e-13, atol=1e-13)


def test_member_permutation_and_duplication_invariance():
    Z = _rand(7, 5, 64, scale=0.5)
    X = _rand(8, 9, 64, scale=0.5)
    t = 0.6
    S = ensf.prior_score(Z, X, t)
    perm = np.random.default_rng(0).permutation(9)
    np.testing.assert_allclose(ensf.prior_score(Z, X[perm], t), S, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(ensf.prior_score(Z, np.vstack([X, X]), t), S, rtol=1e-12,
                               atol=1e-12)


def test_two_member_closed_form():
    # two members: w_1 = sigmoid((|z - a x2|^2 - |z - a x1|^2) / (2 beta^2))
    rng = np.random.default_rng(9)
    z, x1, x2 = rng.standard_normal((3, 7)) * 0.4
    t = 0.4
    a = ensf.schedule(t)["alpha"]
    d1 = np.sum((z - a * x1) ** 2)
    d2 = np.sum((z - a * x2) ** 2)
    w1 = 1.0 / (1.0 + np.exp((d1 - d2) / (2 * t)))
    want = -(z - a * (w1 * x1 + (1 - w1) * x2)) / t
    np.testing.assert_allclose(ensf.prior_score(z[None], np.stack([x1, x2]), t)[0], want,
                               rtol=1e-12)


@pytest.mark.parametrize("op", ["arctan", "linear"])
def test_likelihood_score_is_gradient_of_log_likelihood(op):
    rng = np.random.default_rng(10)
    d = 6
    idx = np.array([0, 2, 2, 5])           # duplicate index: two independent factors
    y = rng.standard_normal(idx.size) * 0.5
    sig = 0.3
    z = rng.standard_normal(d)
    A, B = ensf.densify(idx, y, d, sig)
    g = ensf.likelihood_score(z[None], A, B, op)[0]
    fd = np.zeros(d)
    hstep = 1e-5
    for e in range(d):
        zp, zm = z.copy(), z.copy()
        zp[e] += hstep
        zm[e] -= hstep
        fd[e] = (ensf.log_likelihood(zp, idx, y, sig, op)
                 - ensf.log_likelihood(zm, idx, y, sig, op)) / (2 * hstep)
    np.testing.assert_allclose(g, fd, rtol=1e-8, atol=1e-8)
    assert g[1] == 0 and g[3] == 0 and g[4] == 0


@pytest.mark.parametrize("t", [0.999, 0.7, 0.3, 0.05])
def test_schedule_matches_numerical_derivatives(t):
    eps = 0.05
    dlt = 1e-6
    s = ensf.schedule(t, eps)
    la = lambda u: np.log(1.0 - u * (1.0 - eps))
    b_fd = (la(t + dlt) - la(t - dlt)) / (2 * dlt)
    assert abs(s["b"] - b_fd) <= 1e-8 * abs(b_fd)
    dbeta2 = ((t + dlt) - (t - dlt)) / (2 * dlt)
    assert abs(s["sigma2"] - (dbeta2 - 2 * b_fd * t)) <= 1e-8 * s["sigma2"]
    assert s["h"] == pytest.approx(1 - t)
    # the forward SDE's marginal at t must be N(alpha z0, beta^2): the variance ODE
    # dV/dt = 2 b V + sigma^2 with V(0) = 0 is solved by V = beta^2 = t
    assert abs(2 * s["b"] * t + s["sigma2"] - 1.0) < 1e-12


def test_forward_marginal_from_schedule_integration():
    # integrate the forward SDE moment equations (eq. 6) with the schedule of eq. 9:
    # m' = b m, V' = 2 b V + sigma^2; they must reproduce alpha_t z0 and beta_t^2
    eps = 0.05
    n = 20000
    dt = 1.0 / n
    m, V = 1.0, 0.0
    for k in range(n):
        t = (k + 0.5) * dt
        s = ensf.schedule(t, eps)
        m += s["b"] * m * dt
        V += (2 * s["b"] * V + s["sigma2"]) * dt
    assert abs(m - (1 - (1 - eps))) < 1e-4
    assert abs(V - 1.0) < 1e-4


def test_particle_subset_independence():
    rng = np.random.default_rng(11)
    X = rng.standard_normal((6, 40))
    idx = np.arange(0, 40, 3)
    y = np.arctan(rng.standard_normal(idx.size))
    full = ensf.analysis(X, idx, y, 0.5, 30, seed=99, filter_id=2, n_particles=8)
    sub = ensf.analysis(X, idx, y, 0.5, 30, seed=99, filter_id=2, particle_ids=[1, 6])
    np.testing.assert_allclose(sub, full[[1, 6]], rtol=1e-12, atol=1e-12)


def test_no_observation_run_is_prior_resampling_bias_free():
    # with no observations and a one-member ensemble the exact marginal is tracked:
    # the scheme must contract the particles onto alpha x as t -> 0
    x = np.full((1, 512), 0.7)
    Z = ensf.analysis(x, np.zeros(0, dtype=int), np.zeros(0), 1.0, 400, seed=5)
    # final step pulls z to alpha_{dt} x plus O(sqrt(dt)) noise
    assert abs(Z.mean() - 0.7) < 0.02
    assert Z.std() < 0.2


def test_relax_spread_restores_prior_spread():
    rng = np.random.default_rng(12)
    X = rng.standard_normal((30, 50)) * 2.0
    Z = rng.standard_normal((40, 50)) * 0.3 + 1.0
    R = ensf.relax_spread(Z, X, 1.0)
    np.testing.assert_allclose(R.std(axis=0, ddof=1), X.std(axis=0, ddof=1), rtol=1e-12)
    np.testing.assert_allclose(R.mean(axis=0), Z.mean(axis=0), rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(ensf.relax_spread(Z, X, 0.0), Z)


def test_rel_l2():
    assert ensf.rel_l2([1.0, 0.0], [1.0, 0.0]) == 0.0
    assert ensf.rel_l2([0.0, 1.0], [1.0, 0.0]) == pytest.approx(np.sqrt(2))
