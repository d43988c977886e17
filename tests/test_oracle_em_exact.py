"""Exact pin of the oracle's Euler-Maruyama loop (eq. 7) with no Monte-Carlo score error.

With one forecast member x the Monte-Carlo prior score of eq. 15 is exactly the score of
the diffused law N(alpha x, beta^2) (eq. 12 with a point-mass prior), so the posterior
score of eq. 17 with an identity observation is affine in z and every particle component
is exactly Gaussian, with the mean m and variance v of the closed-form recursion of
`oracle.linear_gaussian` (prior variance s2 = 0).  Components with the same member value
and observation are i.i.d. across components and particles, so pooling P x d/2 of them
pins (m, v) to a plain 4-sigma band (mean) and chi-square band (variance), with no
additive allowance.

The same statistics with a slip planted in the oracle (a shifted time grid, a 3 % error in
the drift, no noise on the last step) land tens to hundreds of standard errors away: the
pin sees each of them.
"""
import numpy as np
import pytest

from oracle import ensf
from oracle import linear_gaussian as lg

D_HALF = 16384
MU, Y = 1.0, -1.0      # member value and observed value (observation far from the prior)


def _z_scores(lik_step, sigma_o, K, n_particles, seed):
    """Runs the oracle on one member with every other component observed and returns the
    (mean, variance) z-scores of the observed and the unobserved group."""
    d = 2 * D_HALF
    X = np.full((1, d), MU)
    idx = np.arange(0, d, 2)
    Z = ensf.analysis(X, idx, np.full(idx.size, Y), sigma_o, K, seed=seed, obs_op="linear",
                      n_particles=n_particles, chunk=n_particles, lik_step=lik_step)
    out = []
    for group, (A, B) in ((Z[:, 0::2], (Y / sigma_o ** 2, 1.0 / sigma_o ** 2)),
                          (Z[:, 1::2], (0.0, 0.0))):
        m, v = lg.em_recursion(MU, 0.0, A, B, K, lik_step=lik_step)
        n = group.size
        zm = (group.mean() - m) / np.sqrt(v / n)
        zv = (group.var(ddof=1) / v - 1.0) / np.sqrt(2.0 / (n - 1))
        print(f"mean {group.mean():.6f} vs {m:.6f} (z {zm:+.2f}); "
              f"var {group.var(ddof=1):.6e} vs {v:.6e} (z {zv:+.2f})")
        out += [zm, zv]
    return np.array(out)


@pytest.mark.parametrize("lik_step,sigma_o,K", [("explicit", 0.3, 100), ("implicit", 0.05, 100),
                                                ("explicit", 0.5, 37)])
def test_one_member_statistics_equal_recursion(lik_step, sigma_o, K):
    z = _z_scores(lik_step, sigma_o, K, n_particles=32,
                  seed=2024 + K + (7 if lik_step == "implicit" else 0))
    assert np.all(np.abs(z) < 4.0), z


def _shifted_grid(monkeypatch, K):
    # scores evaluated on the grid of K + 1 points, t = 1 - k / (K + 1), with the step
    # still 1 / K
    orig = ensf.schedule
    monkeypatch.setattr(ensf, "schedule",
                        lambda t, eps=0.05: orig(1.0 - (1.0 - t) * K / (K + 1.0), eps))


def _drift_error(monkeypatch, K):
    # b and sigma^2 of eq. 9 both 3 % small (the drift b z - sigma^2 s and the noise)
    orig = ensf.schedule

    def sched(t, eps=0.05):
        s = dict(orig(t, eps))
        s["b"] *= 0.97
        s["sigma2"] *= 0.97
        return s
    monkeypatch.setattr(ensf, "schedule", sched)


def _no_last_noise(monkeypatch, K):
    orig = ensf.philox.normals

    def normals(seed, filter_id, step, particles, n):
        out = orig(seed, filter_id, step, particles, n)
        return out * 0.0 if step == K - 1 else out
    monkeypatch.setattr(ensf.philox, "normals", normals)


@pytest.mark.parametrize("slip", [_shifted_grid, _drift_error, _no_last_noise])
def test_pin_rejects_planted_slips(monkeypatch, slip):
    K = 100
    slip(monkeypatch, K)
    z = _z_scores("explicit", 0.3, K, n_particles=16, seed=99)
    assert np.max(np.abs(z)) > 8.0, z


def test_first_step_has_no_likelihood():
    # h(t) = 1 - t vanishes at t = 1: with K = 1 the only step is taken there, so the
    # observations cannot move the particles at all
    rng = np.random.default_rng(5)
    X = rng.standard_normal((4, 24))
    idx = np.arange(0, 24, 3)
    a = ensf.analysis(X, idx, rng.standard_normal(idx.size), 0.2, 1, seed=3, n_particles=5,
                      obs_op="linear")
    b = ensf.analysis(X, np.zeros(0, dtype=np.int64), np.zeros(0), 0.2, 1, seed=3,
                      n_particles=5, obs_op="linear")
    np.testing.assert_array_equal(a, b)
