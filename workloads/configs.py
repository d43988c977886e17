"""Seeded analysis problems with the shapes of the five benchmark configurations.

Each problem is a prior ensemble X (N x d, float32, row-major), a truth, and a set of
observations (sorted int32 indices into the state, float32 values, noise std sigma_o).
Members are the truth plus an independent smooth field ("drawn around a seeded truth").
Observed values are h(truth) plus Gaussian noise with h = arctan (the nonlinear operator)
or the identity (the paper's own twin experiment, Sec. IV-A).

Seeds: data_seed = 2407 + config number drives numpy's PCG64 for every draw here;
the filter's own counter-based noise uses seed = 12168 + config number.
"""
import os
from dataclasses import dataclass, field

import numpy as np

from .fields import smooth_fields

CONFIG_SEEDS = {c: (2407 + c, 12168 + c) for c in range(1, 6)}


@dataclass
class Problem:
    X: np.ndarray            # (N, d) float32
    truth: np.ndarray        # (d,) float64
    obs_idx: np.ndarray      # (m,) int32, sorted
    obs_val: np.ndarray      # (m,) float32
    sigma_o: float
    n_steps: int
    seed: int
    filter_id: int = 0
    obs_op: str = "arctan"
    shape: tuple = ()        # (levels, h, w)
    meta: dict = field(default_factory=dict)

    @property
    def n_members(self):
        return self.X.shape[0]

    @property
    def dim(self):
        return self.X.shape[1]


def _obs_indices(rng, levels, h, w, obs_fraction=None, obs_stride=None):
    d = levels * h * w
    if obs_stride is not None:
        lv, iy, ix = np.meshgrid(np.arange(levels), np.arange(0, h, obs_stride),
                                 np.arange(0, w, obs_stride), indexing="ij")
        return np.sort((lv * h * w + iy * w + ix).reshape(-1)).astype(np.int32)
    if obs_fraction is None or obs_fraction >= 1.0:
        return np.arange(d, dtype=np.int32)
    m = max(1, int(round(obs_fraction * d)))
    return np.sort(rng.choice(d, size=m, replace=False)).astype(np.int32)


def make_problem(levels, h, w, n_members, sigma_o, n_steps, data_seed, seed,
                 obs_fraction=1.0, obs_stride=None, obs_op="arctan", filter_id=0,
                 member_spread=1.0):
    rng = np.random.default_rng(data_seed)
    truth = smooth_fields(rng, levels, h, w).reshape(-1)
    pert = smooth_fields(rng, n_members * levels, h, w).reshape(n_members, -1)
    X = (truth[None, :] + member_spread * pert).astype(np.float32)
    idx = _obs_indices(rng, levels, h, w, obs_fraction, obs_stride)
    clean = np.arctan(truth[idx]) if obs_op == "arctan" else truth[idx]
    y = (clean + sigma_o * rng.standard_normal(idx.size)).astype(np.float32)
    return Problem(X=X, truth=truth, obs_idx=idx, obs_val=y, sigma_o=float(sigma_o),
                   n_steps=int(n_steps), seed=int(seed), filter_id=int(filter_id),
                   obs_op=obs_op, shape=(levels, h, w))


def config_shapes(c):
    """(levels, h, w, N, sigma_o, K, obs_fraction, obs_stride) of configuration c."""
    return {
        1: (2, 64, 64, 20, 0.05, 100, 1.0, None),
        2: (2, 128, 128, 256, 0.05, 100, 0.25, None),
        3: (2, 256, 256, 1024, 0.02, 200, 1.0, None),
        5: (2, 128, 128, 512, 0.05, 400, None, 4),
    }[c]


def config_problem(c, n_steps=None, n_members=None, obs_op="arctan"):
    levels, h, w, N, sig, K, frac, stride = config_shapes(c)
    data_seed, seed = CONFIG_SEEDS[c]
    return make_problem(levels, h, w, n_members or N, sig,
                        n_steps if n_steps is not None else K, data_seed, seed,
                        obs_fraction=frac, obs_stride=stride, obs_op=obs_op)


def batched_problems(n_filters=64, n_steps=100, sigma_o=0.05, data_seed=2411, seed=12172,
                     dims=((2, 64, 64), (2, 128, 128), (2, 256, 256)), n_range=(32, 512),
                     frac_range=(0.1, 1.0)):
    """Independent filters of uneven size: d uniform over `dims`, N uniform over
    n_range (inclusive), observed fraction uniform over frac_range."""
    rng = np.random.default_rng(data_seed)
    specs = []
    for f in range(n_filters):
        levels, h, w = dims[rng.integers(len(dims))]
        N = int(rng.integers(n_range[0], n_range[1] + 1))
        frac = float(rng.uniform(*frac_range))
        sub_seed = int(rng.integers(1 << 31))
        specs.append((levels, h, w, N, frac, sub_seed, f))
    # each filter has its own seed, so drawing them concurrently is deterministic
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(max_workers=max(1, min(8, os.cpu_count() or 1))) as ex:
        return list(ex.map(lambda sp: make_problem(sp[0], sp[1], sp[2], sp[3], sigma_o, n_steps,
                                                   sp[5], seed, obs_fraction=sp[4],
                                                   filter_id=sp[6]), specs))
