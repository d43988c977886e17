"""Pins of the oracle's linearly implicit likelihood step (a variant of the Euler-Maruyama
step of eq. 7 in which the damped likelihood drift is divided by 1 + sigma^2 h kappa dt,
kappa the Gauss-Newton curvature of -log p): the closed-form mean/variance recursion for a
Gaussian prior and a linear observation, exact agreement with the explicit step where
nothing is observed, first-order convergence to the explicit step as dt -> 0, and
insensitivity of whole trajectories at the literal pseudo-step counts where the explicit
step is chaotic."""
import numpy as np
import pytest

import workloads
from oracle import ensf
from oracle import linear_gaussian as lg

from test_oracle_linear_gaussian import quantile_members


@pytest.mark.parametrize("sigma_o,y,K,seed", [(0.05, 0.8, 100, 11), (0.1, -0.4, 50, 12)])
def test_implicit_particles_follow_discrete_recursion(sigma_o, y, K, seed):
    # dt >= sigma_o^2 here: the explicit scheme diverges, the implicit one must not.
    # Members at the normal quantiles (see test_oracle_linear_gaussian): no allowance
    # beyond the particles' own sampling error.
    N, P = 2048, 1024
    X = quantile_members(0.3, N)
    Z = ensf.analysis(X, np.array([0]), np.array([y]), sigma_o, K, seed=seed, obs_op="linear",
                      n_particles=P, chunk=256, lik_step="implicit")
    mh, s2h = X[:, 0].mean(), X[:, 0].var(ddof=1)
    m, v = lg.em_recursion(mh, s2h, y / sigma_o ** 2, 1.0 / sigma_o ** 2, K, lik_step="implicit")
    print(f"particles {Z[:, 0].mean():.4f} / {Z[:, 0].var(ddof=1):.5f}, "
          f"recursion {m:.4f} / {v:.5f}")
    assert abs(Z[:, 0].mean() - m) < 4 * np.sqrt(v / P)
    assert abs(Z[:, 0].var(ddof=1) / v - 1.0) < 4 * np.sqrt(2.0 / (P - 1))


def test_implicit_recursion_stable_where_explicit_diverges():
    s2o = 0.0025
    m_exp, _ = lg.em_recursion(0.0, 1.0, 1.0 / s2o, 1.0 / s2o, 100)
    m_imp, _ = lg.em_recursion(0.0, 1.0, 1.0 / s2o, 1.0 / s2o, 100, lik_step="implicit")
    m_ref, _ = lg.em_recursion(0.0, 1.0, 1.0 / s2o, 1.0 / s2o, 20000)
    assert abs(m_exp) > 1e3
    assert abs(m_imp - m_ref) < 1e-3


def test_implicit_equals_explicit_without_observations():
    rng = np.random.default_rng(3)
    X = rng.standard_normal((7, 33))
    none = np.zeros(0, dtype=np.int64)
    a = ensf.analysis(X, none, np.zeros(0), 0.3, 40, seed=5, n_particles=9)
    b = ensf.analysis(X, none, np.zeros(0), 0.3, 40, seed=5, n_particles=9, lik_step="implicit")
    np.testing.assert_allclose(b, a, rtol=0, atol=1e-12)


@pytest.mark.parametrize("obs_op", ["arctan", "linear"])
def test_implicit_converges_to_explicit_first_order(obs_op):
    # same noise, same K: the two schemes differ by O(dt^2) per step, so the difference must
    # shrink at least linearly in dt (measured: about quadratically)
    rng = np.random.default_rng(4)
    X = rng.standard_normal((6, 40))
    idx = np.arange(0, 40, 2)
    y = np.arctan(rng.standard_normal(idx.size)) if obs_op == "arctan" else rng.standard_normal(idx.size)
    diffs = []
    for K in (200, 400, 800):
        a = ensf.analysis(X, idx, y, 0.7, K, seed=9, n_particles=64, obs_op=obs_op)
        b = ensf.analysis(X, idx, y, 0.7, K, seed=9, n_particles=64, obs_op=obs_op,
                          lik_step="implicit")
        diffs.append(np.sqrt(np.mean((a - b) ** 2)))
    print(obs_op, diffs)
    assert diffs[0] < 0.05
    assert diffs[1] / diffs[0] < 0.6 and diffs[2] / diffs[1] < 0.6


@pytest.mark.parametrize("config,rows", [(1, None), (2, [0, 255])])
def test_literal_k_trajectories_are_pinnable_with_implicit_step(config, rows):
    # the stability gate: a 1e-12 relative change of the prior must stay below 1e-9 after
    # the whole analysis at the workload's own K; the explicit step amplifies it to O(1)
    p = workloads.config_problem(config)
    Xp = p.X.astype(np.float64) * (1.0 + 1e-12)
    kw = dict(particle_ids=rows) if rows else {}
    a = ensf.analysis(p.X, p.obs_idx, p.obs_val, p.sigma_o, p.n_steps, p.seed,
                      lik_step="implicit", **kw)
    b = ensf.analysis(Xp, p.obs_idx, p.obs_val, p.sigma_o, p.n_steps, p.seed,
                      lik_step="implicit", **kw)
    e_imp = ensf.rel_l2(b, a)
    c = ensf.analysis(p.X, p.obs_idx, p.obs_val, p.sigma_o, p.n_steps, p.seed, **kw)
    d = ensf.analysis(Xp, p.obs_idx, p.obs_val, p.sigma_o, p.n_steps, p.seed, **kw)
    e_exp = ensf.rel_l2(d, c)
    print(f"c{config} K={p.n_steps}: implicit sensitivity {e_imp:.2e}, explicit {e_exp:.2e}")
    assert e_imp <= 1e-9
    assert e_exp > 1e-3
