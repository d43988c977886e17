"""GPU parity of the HIP path (through the C ABI) against the FP64 oracle.

Tolerances (rel-L2 = ||gpu - oracle|| / ||oracle||):
  score at fixed t          FP32 <= 2e-5, split BF16 <= 2e-4   (one evaluation, no chaos)
  posterior mean, stable K  <= 1e-3 (FP32 and split BF16)       (the filter's accuracy bar)
  ragged small problem      elementwise, max |diff| <= 5e-4 * max |oracle|
Trajectories are compared only at pseudo-step counts where explicit Euler-Maruyama is
contractive (K >= 1/sigma_o^2); at smaller K the discrete map is chaotic and a 1e-12
perturbation of the input already changes the result at O(0.1).
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import workloads
from oracle import ensf as O
from oracle import philox
from paper_2407_12168_amd import ensf

pytestmark = pytest.mark.gpu

SCORE_TOL = {"fp32": 2e-5, "bf16x3": 2e-4}


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _gpu(a, dev, dtype=None):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


def _run(dev, p, precision, n_particles=None, use_graph=True, obs_op=None, spread_relax=0.0):
    X = _gpu(p.X, dev)
    post = torch.empty((n_particles or p.n_members, p.dim), device=dev)
    idx = _gpu(p.obs_idx, dev)
    val = _gpu(p.obs_val, dev)
    with ensf.Context(precision=precision, use_graph=use_graph, obs_op=obs_op or p.obs_op,
                      spread_relax=spread_relax) as ctx:
        ensf.ensf_analysis(ctx.handle, X, post, idx, val, p.sigma_o, p.n_steps, p.seed,
                           p.filter_id)
        st, nbad = ensf.ensf_sync_status(ctx.handle)
    assert st == ensf.ENSF_OK, (st, nbad)
    return post.cpu().numpy().astype(np.float64)


# ---------------------------------------------------------------------------------------
# counter-based generator

def test_rng_raw_words_bit_exact_and_normals(dev):
    n = 1003
    for (seed, filt, step, part) in [(12168, 0, 0, 0), (2**40 + 5, 7, 399, 1023),
                                     (1, 3, philox.INIT_STEP, 9)]:
        out = torch.empty(n, device=dev)
        raw = torch.empty(4 * ((n + 3) // 4), dtype=torch.int32, device=dev)
        ensf.ensf_rng_normal(seed, filt, step, part, out, raw)
        torch.cuda.synchronize()
        want_raw = philox.raw_words(seed, filt, step, [part], n)[0].reshape(-1)
        np.testing.assert_array_equal(raw.cpu().numpy().view(np.uint32), want_raw.astype(np.uint32))
        want = philox.normals(seed, filt, step, [part], n)[0]
        np.testing.assert_allclose(out.cpu().numpy(), want, rtol=2e-6, atol=2e-6)


# ---------------------------------------------------------------------------------------
# score at fixed pseudo-time: the well-posed check at every configuration's shape

def _score_case(dev, p, t, precision, n_particles, rows=None):
    rng = np.random.default_rng(123)
    s = O.schedule(t)
    pick = rng.integers(0, p.n_members, n_particles)
    Z = (s["alpha"] * p.X[pick].astype(np.float64)
         + np.sqrt(s["beta2"]) * rng.standard_normal((n_particles, p.dim))).astype(np.float32)
    Xg, Zg = _gpu(p.X, dev), _gpu(Z, dev)
    score = torch.empty_like(Zg)
    W = torch.empty((n_particles, p.n_members), device=dev)
    with ensf.Context(precision=precision, obs_op=p.obs_op) as ctx:
        ensf.ensf_score(ctx.handle, Xg, Zg, _gpu(p.obs_idx, dev), _gpu(p.obs_val, dev),
                        p.sigma_o, t, score, W)
        torch.cuda.synchronize()
    rows = np.arange(n_particles) if rows is None else np.asarray(rows)
    A, B = O.densify(p.obs_idx, p.obs_val, p.dim, p.sigma_o)
    Zr = Z[rows].astype(np.float64)
    Xd = p.X.astype(np.float64)
    want = O.posterior_score(Zr, Xd, A, B, t, obs_op=p.obs_op)
    want_w = O.prior_weights(Zr, Xd, t)
    got = score.cpu().numpy()[rows].astype(np.float64)
    got_w = W.cpu().numpy()[rows].astype(np.float64)
    return O.rel_l2(got, want), np.abs(got_w - want_w).max(), np.abs(got_w.sum(1) - 1).max()


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
@pytest.mark.parametrize("t", [1.0, 0.5, 0.1, 0.0025])
def test_score_parity_config1_shape(dev, precision, t):
    p = workloads.config_problem(1)
    err, werr, wsum = _score_case(dev, p, t, precision, p.n_members)
    print(f"c1 score {precision} t={t}: rel-L2 {err:.2e}, max|dw| {werr:.2e}")
    assert err <= SCORE_TOL[precision]
    assert wsum <= 1e-5


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
@pytest.mark.parametrize("t", [1.0, 0.1, 0.01])
def test_score_parity_config2_shape(dev, precision, t):
    p = workloads.config_problem(2)
    err, werr, wsum = _score_case(dev, p, t, precision, p.n_members, rows=[0, 1, 100, 255])
    print(f"c2 score {precision} t={t}: rel-L2 {err:.2e}, max|dw| {werr:.2e}")
    assert err <= SCORE_TOL[precision]
    assert wsum <= 1e-5


@pytest.mark.parametrize("t", [0.5, 0.01])
def test_split_form_recovers_what_plain_bf16_loses(dev, t):
    """The three forms on the same c2-shape score evaluation: plain BF16 operands (one product)
    lose the cancellation in |x_j|^2 - 2 alpha x_j.x_k + alpha^2 |x_k|^2, amplified by 1/beta^2
    in the logits; the split form (hi.hi + hi.lo + lo.hi) stays at FP32-level error."""
    p = workloads.config_problem(2)
    rows = [0, 1, 100, 255]
    errs = {f: _score_case(dev, p, t, f, p.n_members, rows=rows)[0]
            for f in ("fp32", "bf16x3", "bf16")}
    print(f"c2 score t={t}: rel-L2 fp32 {errs['fp32']:.2e}, split {errs['bf16x3']:.2e}, "
          f"plain BF16 {errs['bf16']:.2e}")
    assert errs["bf16x3"] <= SCORE_TOL["bf16x3"]
    assert errs["bf16"] > 10 * errs["bf16x3"]


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_score_parity_config3_shape_sampled_rows(dev, precision):
    # full size (N = 1024, d = 131072); the oracle checks sampled particle rows
    p = workloads.config_problem(3)
    err, werr, wsum = _score_case(dev, p, 0.5, precision, p.n_members, rows=[0, 511, 1023])
    print(f"c3 score {precision}: rel-L2 {err:.2e}, max|dw| {werr:.2e}")
    assert err <= SCORE_TOL[precision]
    assert wsum <= 1e-5


# ---------------------------------------------------------------------------------------
# full analyses at EM-stable pseudo-step counts

@pytest.fixture(scope="module")
def c1_oracle():
    p = workloads.config_problem(1, n_steps=400)
    return p, O.analysis(p.X, p.obs_idx, p.obs_val, p.sigma_o, p.n_steps, p.seed)


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_trajectory_parity_config1_stable_k(dev, c1_oracle, precision):
    p, want = c1_oracle
    got = _run(dev, p, precision)
    mean_err = O.rel_l2(got.mean(0), want.mean(0))
    sd_err = O.rel_l2(got.std(0, ddof=1), want.std(0, ddof=1))
    elem = np.abs(got - want).max() / np.abs(want).max()
    print(f"c1 K=400 {precision}: mean rel-L2 {mean_err:.2e}, spread rel-L2 {sd_err:.2e}, "
          f"particles {O.rel_l2(got, want):.2e}, max elementwise {elem:.2e}")
    assert mean_err <= 1e-3
    assert sd_err <= 1e-2
    assert O.rel_l2(got, want) <= 1e-3 and elem <= 1e-3


def test_ragged_small_problem_elementwise(dev):
    # N, particles and d not multiples of any tile; duplicate observation indices
    rng = np.random.default_rng(5)
    N, M, d = 5, 7, 1001
    X = rng.standard_normal((N, d)).astype(np.float32)
    idx = np.sort(rng.choice(d, 300, replace=True)).astype(np.int32)
    y = np.arctan(rng.standard_normal(idx.size)).astype(np.float32)
    p = workloads.Problem(X=X, truth=None, obs_idx=idx, obs_val=y, sigma_o=0.5, n_steps=60,
                          seed=77, filter_id=3)
    for precision in ("fp32", "bf16x3"):
        got = _run(dev, p, precision, n_particles=M)
        want = O.analysis(X, idx, y, 0.5, 60, seed=77, filter_id=3, n_particles=M)
        err = np.abs(got - want).max() / np.abs(want).max()
        print(f"ragged {precision}: max rel diff {err:.2e}")
        assert err <= 5e-4


@pytest.fixture(scope="module")
def c2_stable():
    p = workloads.config_problem(2, n_steps=400)
    rows = [0, 77, 255]
    return p, rows, O.analysis(p.X, p.obs_idx, p.obs_val, p.sigma_o, p.n_steps, p.seed,
                               particle_ids=rows)


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_config2_particle_subset_stable_k(dev, c2_stable, precision):
    p, rows, want = c2_stable
    got = _run(dev, p, precision)[rows]
    err = O.rel_l2(got, want)
    elem = np.abs(got - want).max() / np.abs(want).max()
    print(f"c2 K=400 {precision} particles {rows}: rel-L2 {err:.2e}, max elementwise {elem:.2e}")
    assert err <= 1e-3 and elem <= 1e-3


def test_duplicate_observations_deterministic_in_any_order(dev):
    # many observations of the same components, given in two different orders: the
    # densified sums are formed in observation order in FP64 on the device, so both runs
    # (and a repeat) give the same bits, and match the oracle
    rng = np.random.default_rng(17)
    N, M, d = 24, 16, 3000
    X = rng.standard_normal((N, d)).astype(np.float32)
    idx = rng.integers(0, 40, 5000).astype(np.int32)        # ~125 observations per component
    y = (0.3 * rng.standard_normal(idx.size)).astype(np.float32)
    perm = rng.permutation(idx.size)
    runs = []
    for order in (np.arange(idx.size), perm, np.arange(idx.size)):
        p = workloads.Problem(X=X, truth=None, obs_idx=idx[order], obs_val=y[order],
                              sigma_o=3.0, n_steps=60, seed=5)
        runs.append(_run(dev, p, "fp32", n_particles=M))
    np.testing.assert_array_equal(runs[0], runs[2])
    want = O.analysis(X, idx, y, 3.0, 60, seed=5, n_particles=M)
    for got in runs[:2]:
        assert np.abs(got - want).max() <= 5e-4 * np.abs(want).max()
    # the two orders give the same A and B up to the FP64 rounding of the sums, so the
    # particles agree far below the FP32 parity bar
    assert np.abs(runs[0] - runs[1]).max() <= 1e-5 * np.abs(want).max()


def test_calls_on_two_streams_of_one_context_run_in_order(dev):
    # two analyses of different problems on one context, the second on another stream
    # without any host synchronisation in between: the second must wait for the first
    # (they share the context's workspace), so both equal their single-stream results
    pa = workloads.config_problem(1, n_steps=50)
    pb = workloads.make_problem(2, 64, 64, 20, 0.05, 50, data_seed=3, seed=4)
    ref = [_run(dev, q, "fp32") for q in (pa, pb)]
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    outs = []
    with ensf.Context(precision="fp32") as ctx:
        ins = []
        for q in (pa, pb):
            ins.append((_gpu(q.X, dev), torch.empty((q.n_members, q.dim), device=dev),
                        _gpu(q.obs_idx, dev), _gpu(q.obs_val, dev)))
        torch.cuda.synchronize()
        for q, (X, post, idx, val), s in zip((pa, pb), ins, (s1, s2)):
            ensf.ensf_analysis(ctx.handle, X, post, idx, val, q.sigma_o, q.n_steps, q.seed,
                               q.filter_id, s)
        st, nbad = ensf.ensf_sync_status(ctx.handle)
        assert st == ensf.ENSF_OK, (st, nbad)
        outs = [post.cpu().numpy().astype(np.float64) for (_, post, _, _) in ins]
    for got, want in zip(outs, ref):
        np.testing.assert_array_equal(got, want)


def test_deterministic_and_graph_equals_eager(dev):
    p = workloads.config_problem(1, n_steps=50)
    a = _run(dev, p, "bf16x3")
    b = _run(dev, p, "bf16x3")
    c = _run(dev, p, "bf16x3", use_graph=False)
    np.testing.assert_array_equal(a, b)
    np.testing.assert_array_equal(a, c)


# ---------------------------------------------------------------------------------------
# error paths

def test_invalid_arguments_rejected(dev):
    X = torch.zeros((4, 64), device=dev)
    post = torch.zeros((4, 64), device=dev)
    idx = torch.zeros(3, dtype=torch.int32, device=dev)
    val = torch.zeros(3, device=dev)
    L = ensf._lib()
    with ensf.Context() as ctx:
        h = ctx.handle
        s = ensf._stream(None)
        assert L.ensf_analysis(h, X.data_ptr(), 0, 64, post.data_ptr(), 4, None, None, 0,
                               1.0, 10, 1, 0, s) == ensf.ENSF_EINVAL
        assert L.ensf_analysis(h, X.data_ptr(), 4, 64, X.data_ptr(), 4, None, None, 0,
                               1.0, 10, 1, 0, s) == ensf.ENSF_EINVAL      # post aliases prior
        assert L.ensf_analysis(h, X.data_ptr(), 4, 64, post.data_ptr(), 4, idx.data_ptr(),
                               val.data_ptr(), 3, 0.0, 10, 1, 0, s) == ensf.ENSF_EINVAL
        assert L.ensf_analysis(h, X.data_ptr(), 4, 64, post.data_ptr(), 4, None, None, 0,
                               1.0, 0, 1, 0, s) == ensf.ENSF_EINVAL
        assert L.ensf_analysis(h, None, 4, 64, post.data_ptr(), 4, None, None, 0, 1.0, 10, 1,
                               0, s) == ensf.ENSF_EINVAL
        assert ensf.ensf_sync_status(h)[0] == ensf.ENSF_OK


def test_out_of_range_observation_and_nonfinite_reported(dev):
    X = torch.randn((4, 64), device=dev)
    post = torch.zeros((4, 64), device=dev)
    idx = torch.tensor([1, 64], dtype=torch.int32, device=dev)
    val = torch.zeros(2, device=dev)
    with ensf.Context() as ctx:
        ensf.ensf_analysis(ctx.handle, X, post, idx, val, 1.0, 10, 1)
        assert ensf.ensf_sync_status(ctx.handle)[0] == ensf.ENSF_EINVAL
        X[2, 5] = float("nan")
        ensf.ensf_analysis(ctx.handle, X, post, idx[:1], val[:1], 1.0, 10, 1)
        st, n = ensf.ensf_sync_status(ctx.handle)
        assert st == ensf.ENSF_ENONFINITE and n > 0


# ---------------------------------------------------------------------------------------
# Gaussian prior, linear observation, large ensemble: the GPU particles must follow the
# closed-form recursion of the scheme (and the Kalman gap is reported)

def quantile_members_2d(mu, n, seed):
    """n members of N(mu, I_2): both components at the normal quantiles (j + 1/2)/n, the
    second in a seeded random order.  Each component's empirical law is within O(1/n) of
    the Gaussian, so the Monte-Carlo score adds no offset of the size of the particles'
    sampling error; the two components are uncorrelated to O(1/sqrt(n)), which moves the
    unobserved component's mean by about 1e-2 of a standard error here."""
    from scipy.stats import norm
    q = mu + norm.ppf((np.arange(n) + 0.5) / n)
    perm = np.random.default_rng(seed).permutation(n)
    return np.stack([q, q[perm]], axis=1).astype(np.float32)


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_linear_gaussian_large_ensemble(dev, precision):
    from oracle import linear_gaussian as lg
    N, M, K, sig, y = 16384, 4096, 200, 1.0, 1.0
    X = quantile_members_2d(0.3, N, seed=21)
    p = workloads.Problem(X=X, truth=None, obs_idx=np.array([0], np.int32),
                          obs_val=np.array([y], np.float32), sigma_o=sig, n_steps=K, seed=9,
                          obs_op="linear")
    Z = _run(dev, p, precision, n_particles=M, obs_op="linear")
    Xd = X.astype(np.float64)
    for e, (A, B) in enumerate([(y / sig ** 2, 1 / sig ** 2), (0.0, 0.0)]):
        m, v = lg.em_recursion(Xd[:, e].mean(), Xd[:, e].var(ddof=1), A, B, K)
        km, kv = (lg.kalman(Xd[:, e].mean(), Xd[:, e].var(ddof=1), y, sig ** 2) if B
                  else (Xd[:, e].mean(), Xd[:, e].var(ddof=1)))
        print(f"{precision} e{e}: mean {Z[:, e].mean():.4f} recursion {m:.4f} Kalman {km:.4f}; "
              f"var {Z[:, e].var(ddof=1):.4f} recursion {v:.4f} Kalman {kv:.4f}")
        assert abs(Z[:, e].mean() - m) < 4 * np.sqrt(v / M)
        assert abs(Z[:, e].var(ddof=1) / v - 1) < 4 * np.sqrt(2.0 / (M - 1))


def test_no_observations_and_linear_operator_match_oracle(dev):
    rng = np.random.default_rng(8)
    X = rng.standard_normal((9, 300)).astype(np.float32)
    empty = np.zeros(0, np.int32)
    p = workloads.Problem(X=X, truth=None, obs_idx=empty, obs_val=np.zeros(0, np.float32),
                          sigma_o=1.0, n_steps=40, seed=4)
    got = _run(dev, p, "fp32", n_particles=6)
    want = O.analysis(X, empty, np.zeros(0), 1.0, 40, seed=4, n_particles=6)
    assert np.abs(got - want).max() <= 5e-4 * np.abs(want).max()
    idx = np.arange(0, 300, 2).astype(np.int32)
    y = rng.standard_normal(idx.size).astype(np.float32)
    p = workloads.Problem(X=X, truth=None, obs_idx=idx, obs_val=y, sigma_o=0.7, n_steps=40,
                          seed=4, obs_op="linear")
    got = _run(dev, p, "fp32", n_particles=6, obs_op="linear")
    want = O.analysis(X, idx, y, 0.7, 40, seed=4, obs_op="linear", n_particles=6)
    assert np.abs(got - want).max() <= 5e-4 * np.abs(want).max()


def test_ensemble_stats_and_spread_relaxation(dev):
    rng = np.random.default_rng(3)
    E = rng.standard_normal((37, 999)).astype(np.float32)
    mean = torch.empty(999, device=dev)
    sd = torch.empty(999, device=dev)
    ensf.ensf_ensemble_stats(_gpu(E, dev), mean, sd)
    torch.cuda.synchronize()
    m, s = O.posterior_stats(E.astype(np.float64))
    np.testing.assert_allclose(mean.cpu().numpy(), m, rtol=1e-5, atol=1e-6)
    np.testing.assert_allclose(sd.cpu().numpy(), s, rtol=1e-5, atol=1e-6)
    X = (2.0 * rng.standard_normal((12, 256))).astype(np.float32)
    p = workloads.Problem(X=X, truth=None, obs_idx=np.arange(256, dtype=np.int32),
                          obs_val=np.zeros(256, np.float32), sigma_o=0.5, n_steps=30, seed=6)
    got = _run(dev, p, "fp32", spread_relax=1.0)
    want = O.analysis(X, p.obs_idx, p.obs_val, 0.5, 30, seed=6, spread_relax=1.0)
    np.testing.assert_allclose(got.std(0, ddof=1), X.astype(np.float64).std(0, ddof=1),
                               rtol=1e-4)
    assert np.abs(got - want).max() <= 1e-3 * np.abs(want).max()
