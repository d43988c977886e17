"""The synthetic-input recipe: red-spectrum unit-variance fields and observation sets."""
import numpy as np

import workloads


def test_fields_unit_variance_zero_mean_and_slope():
    f = workloads.smooth_fields(np.random.default_rng(0), 3, 128, 128)
    np.testing.assert_allclose(f.mean(axis=(1, 2)), 0.0, atol=1e-12)
    np.testing.assert_allclose(f.std(axis=(1, 2)), 1.0, rtol=1e-12)
    for g in f:
        assert abs(workloads.field_psd_slope(g) + 3.0) < 0.35


def test_config_problems_shapes():
    p = workloads.config_problem(1)
    assert p.X.shape == (20, 8192) and p.X.dtype == np.float32
    assert p.obs_idx.size == 8192 and p.n_steps == 100 and p.sigma_o == 0.05
    p5 = workloads.make_problem(2, 128, 128, 4, 0.05, 400, 1, 2, obs_stride=4)
    assert p5.obs_idx.size == 2048
    p2 = workloads.make_problem(2, 128, 128, 4, 0.05, 100, 1, 2, obs_fraction=0.25)
    assert p2.obs_idx.size == 8192
    assert np.all(np.diff(p2.obs_idx) > 0) and p2.obs_idx.max() < 32768
    np.testing.assert_array_equal(p2.X, workloads.make_problem(2, 128, 128, 4, 0.05, 100, 1, 2,
                                                               obs_fraction=0.25).X)


def test_batched_problem_mix():
    probs = workloads.batched_problems(n_filters=6, dims=((2, 8, 8), (2, 16, 16)), n_range=(3, 9))
    assert len(probs) == 6
    for f, p in enumerate(probs):
        assert p.filter_id == f and 3 <= p.n_members <= 9 and p.dim in (128, 512)
        assert 0.1 * p.dim - 1 <= p.obs_idx.size <= p.dim
