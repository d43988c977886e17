"""GPU parity of the linearly implicit likelihood step (ensf_options.lik_step = IMPLICIT)
against the FP64 oracle's same variant.  With it the whole analysis is contracting at the
workloads' own pseudo-step counts (K = 100 at sigma_o = 0.05, K = 200 at sigma_o = 0.02),
where the explicit step is chaotic, so full trajectories are compared at those K.

Tolerances: rel-L2 of the particles <= 1e-3 (FP32 and split BF16), the filter's bar; the
no-observation case must equal the explicit step bit for bit (the divisor is exactly 1)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import workloads
from oracle import ensf as O
from oracle import linear_gaussian as lg
from paper_2407_12168_amd import ensf

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _run(dev, p, precision, lik_step="implicit", n_particles=None, obs_op=None):
    X = torch.from_numpy(np.ascontiguousarray(p.X)).to(dev)
    post = torch.empty((n_particles or p.n_members, p.dim), device=dev)
    idx = torch.from_numpy(p.obs_idx).to(dev)
    val = torch.from_numpy(p.obs_val).to(dev)
    with ensf.Context(precision=precision, obs_op=obs_op or p.obs_op, lik_step=lik_step) as ctx:
        ensf.ensf_analysis(ctx.handle, X, post, idx, val, p.sigma_o, p.n_steps, p.seed,
                           p.filter_id)
        st, nbad = ensf.ensf_sync_status(ctx.handle)
    assert st == ensf.ENSF_OK, (st, nbad)
    return post.cpu().numpy().astype(np.float64)


@pytest.fixture(scope="module")
def c1_case():
    p = workloads.config_problem(1)          # K = 100, sigma_o = 0.05: the literal count
    return p, O.analysis(p.X, p.obs_idx, p.obs_val, p.sigma_o, p.n_steps, p.seed,
                         lik_step="implicit")


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_literal_k_config1_full_trajectory(dev, c1_case, precision):
    p, want = c1_case
    got = _run(dev, p, precision)
    err = O.rel_l2(got, want)
    mean_err = O.rel_l2(got.mean(0), want.mean(0))
    elem = np.abs(got - want).max() / np.abs(want).max()
    print(f"c1 K={p.n_steps} implicit {precision}: particles rel-L2 {err:.2e}, mean {mean_err:.2e}, "
          f"max elementwise {elem:.2e}")
    assert err <= 1e-3 and mean_err <= 1e-3 and elem <= 1e-3


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_literal_k_config2_particle_subset(dev, precision):
    p = workloads.config_problem(2)          # K = 100, 25 % observed
    got = _run(dev, p, precision)
    rows = [0, 131, 255]
    want = O.analysis(p.X, p.obs_idx, p.obs_val, p.sigma_o, p.n_steps, p.seed,
                      particle_ids=rows, lik_step="implicit")
    err = O.rel_l2(got[rows], want)
    elem = np.abs(got[rows] - want).max() / np.abs(want).max()
    print(f"c2 K={p.n_steps} implicit {precision} particles {rows}: rel-L2 {err:.2e}, "
          f"max elementwise {elem:.2e}")
    assert err <= 1e-3 and elem <= 1e-3


def test_implicit_linear_gaussian_where_explicit_diverges(dev):
    from test_gpu_parity import quantile_members_2d
    N, M, K, sig, y = 16384, 4096, 100, 0.05, 0.8
    X = quantile_members_2d(0.3, N, seed=31)
    p = workloads.Problem(X=X, truth=None, obs_idx=np.array([0], np.int32),
                          obs_val=np.array([y], np.float32), sigma_o=sig, n_steps=K, seed=5,
                          obs_op="linear")
    Z = _run(dev, p, "fp32", n_particles=M, obs_op="linear")
    Xd = X.astype(np.float64)
    for e, (A, B) in enumerate([(y / sig ** 2, 1 / sig ** 2), (0.0, 0.0)]):
        m, v = lg.em_recursion(Xd[:, e].mean(), Xd[:, e].var(ddof=1), A, B, K,
                               lik_step="implicit")
        print(f"e{e}: mean {Z[:, e].mean():.4f} recursion {m:.4f}; var "
              f"{Z[:, e].var(ddof=1):.5f} recursion {v:.5f}")
        assert abs(Z[:, e].mean() - m) < 4 * np.sqrt(v / M)
        assert abs(Z[:, e].var(ddof=1) / v - 1) < 4 * np.sqrt(2.0 / (M - 1))


def test_implicit_equals_explicit_without_observations(dev):
    rng = np.random.default_rng(6)
    X = rng.standard_normal((17, 1000)).astype(np.float32)
    empty = np.zeros(0, np.int32)
    p = workloads.Problem(X=X, truth=None, obs_idx=empty, obs_val=np.zeros(0, np.float32),
                          sigma_o=0.05, n_steps=30, seed=8)
    for precision in ("fp32", "bf16x3"):
        a = _run(dev, p, precision, lik_step="explicit", n_particles=11)
        b = _run(dev, p, precision, lik_step="implicit", n_particles=11)
        np.testing.assert_array_equal(a, b)


def test_invalid_lik_step_rejected(dev):
    with pytest.raises(ensf.EnsfError):
        ensf.Context(lik_step=2)


def test_literal_k_config4_full_batch_sampled(dev):
    # all 64 filters in one batched call, the tuned launch configuration the benchmark
    # times; three filters (largest, smallest, a middle one) checked on two particles each
    probs = workloads.batched_problems(n_filters=64, n_steps=100, sigma_o=0.05)
    tens, descs = [], []
    for p in probs:
        X = torch.from_numpy(p.X).to(dev)
        post = torch.empty_like(X)
        idx = torch.from_numpy(p.obs_idx).to(dev)
        val = torch.from_numpy(p.obs_val).to(dev)
        tens.append((X, post, idx, val))
        descs.append(ensf.make_problem(X, post, idx, val, p.sigma_o, p.n_steps, p.seed,
                                       p.filter_id))
    with ensf.Context(precision="bf16x3", lik_step="implicit") as ctx:
        ensf.ensf_analysis_batched(ctx.handle, descs)
        st, nbad = ensf.ensf_sync_status(ctx.handle)
    assert st == ensf.ENSF_OK, (st, nbad)
    work = [p.n_members ** 2 * p.dim for p in probs]
    order = np.argsort(work)
    for f in (order[-1], order[0], order[len(order) // 2]):
        p = probs[f]
        rows = [0, p.n_members - 1]
        got = tens[f][1][rows].cpu().numpy().astype(np.float64)
        want = O.analysis(p.X, p.obs_idx, p.obs_val, p.sigma_o, p.n_steps, p.seed,
                          filter_id=p.filter_id, particle_ids=rows, lik_step="implicit",
                          chunk=2)
        err = O.rel_l2(got, want)
        print(f"c4 filter {f} (N={p.n_members}, d={p.dim}) particles {rows}: rel-L2 {err:.2e}")
        assert err <= 1e-3
