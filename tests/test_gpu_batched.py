"""Batched form: many independent filters of uneven size in one grouped launch per phase.
Each filter must match the FP64 oracle run alone, and a reused (captured) pseudo-time
graph must pick up new problem descriptors."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import workloads
from oracle import ensf as O
from paper_2407_12168_amd import ensf

pytestmark = pytest.mark.gpu

# (members N, dim d, particles M_p, K, sigma_o, observed fraction)
SPECS = [(5, 300, 7, 40, 0.5, 1.0), (33, 1000, 33, 60, 0.5, 0.3), (64, 2048, 40, 30, 0.5, 0.6),
         (7, 129, 9, 50, 0.5, 1.0), (130, 517, 130, 25, 0.7, 0.2)]


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _problems(seed_base=1000):
    out = []
    for f, (N, d, M, K, sig, frac) in enumerate(SPECS):
        rng = np.random.default_rng(seed_base + f)
        X = rng.standard_normal((N, d)).astype(np.float32)
        m = max(1, int(frac * d))
        idx = np.sort(rng.choice(d, m, replace=False)).astype(np.int32)
        y = np.arctan(rng.standard_normal(m)).astype(np.float32)
        out.append(dict(X=X, idx=idx, y=y, sig=sig, K=K, M=M, seed=seed_base + 7 * f, fid=f))
    return out


def _run_batched(dev, probs, precision, ctx=None):
    tens = []
    descs = []
    for p in probs:
        X = torch.from_numpy(p["X"]).to(dev)
        post = torch.empty((p["M"], p["X"].shape[1]), device=dev)
        idx = torch.from_numpy(p["idx"]).to(dev)
        y = torch.from_numpy(p["y"]).to(dev)
        tens.append((X, post, idx, y))
        descs.append(ensf.make_problem(X, post, idx, y, p["sig"], p["K"], p["seed"], p["fid"]))
    own = ctx is None
    if own:
        ctx = ensf.Context(precision=precision)
    ensf.ensf_analysis_batched(ctx.handle, descs)
    st, nbad = ensf.ensf_sync_status(ctx.handle)
    if own:
        ctx.destroy()
    assert st == ensf.ENSF_OK, (st, nbad)
    return [t[1].cpu().numpy().astype(np.float64) for t in tens]


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_batched_uneven_filters_match_oracle(dev, precision):
    probs = _problems()
    got = _run_batched(dev, probs, precision)
    for p, g in zip(probs, got):
        want = O.analysis(p["X"], p["idx"], p["y"], p["sig"], p["K"], p["seed"], p["fid"],
                          n_particles=p["M"])
        err = np.abs(g - want).max() / np.abs(want).max()
        print(f"{precision} filter {p['fid']} N={p['X'].shape[0]} d={p['X'].shape[1]} "
              f"M={p['M']} K={p['K']}: max rel diff {err:.2e}")
        assert err <= 5e-4


def test_reused_graph_picks_up_new_descriptors(dev):
    a = _problems(1000)
    b = _problems(2000)  # same shapes, new data and seeds
    with ensf.Context(precision="fp32") as ctx:
        _run_batched(dev, a, "fp32", ctx)
        reused = _run_batched(dev, b, "fp32", ctx)
    fresh = _run_batched(dev, b, "fp32")
    for r, f in zip(reused, fresh):
        np.testing.assert_array_equal(r, f)


def test_batched_config4_shapes_small_sample(dev):
    # the uneven-size mix of the 64-filter workload at reduced grid sizes and count
    probs = workloads.batched_problems(n_filters=8, n_steps=30, sigma_o=0.5,
                                       dims=((2, 8, 8), (2, 16, 16), (2, 32, 32)),
                                       n_range=(8, 64))
    ps = [dict(X=p.X, idx=p.obs_idx, y=p.obs_val, sig=p.sigma_o, K=p.n_steps, M=p.n_members,
               seed=p.seed, fid=p.filter_id) for p in probs]
    got = _run_batched(dev, ps, "bf16x3")
    for p, g in zip(ps, got):
        want = O.analysis(p["X"], p["idx"], p["y"], p["sig"], p["K"], p["seed"], p["fid"])
        assert np.abs(g - want).max() <= 5e-4 * np.abs(want).max()


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_batched_autotune_then_match_oracle(dev, precision, tmp_path):
    # the batch tuner records an entry under the batch key; the tuned batch still matches
    probs = _problems(3000)
    cache = tmp_path / "tune.json"
    tens, descs = [], []
    for p in probs:
        X = torch.from_numpy(p["X"]).to(dev)
        post = torch.empty((p["M"], p["X"].shape[1]), device=dev)
        idx = torch.from_numpy(p["idx"]).to(dev)
        y = torch.from_numpy(p["y"]).to(dev)
        tens.append((X, post, idx, y))
        descs.append(ensf.make_problem(X, post, idx, y, p["sig"], p["K"], p["seed"], p["fid"]))
    with ensf.Context(precision=precision, tune_cache=str(cache)) as ctx:
        ensf.ensf_autotune_batched(ctx.handle, descs)
        torch.cuda.synchronize()
        assert "/b2/" in cache.read_text()   # 5 problems -> batch bucket 2
        got = _run_batched(dev, probs, precision, ctx)
    for p, g in zip(probs, got):
        want = O.analysis(p["X"], p["idx"], p["y"], p["sig"], p["K"], p["seed"], p["fid"],
                          n_particles=p["M"])
        assert np.abs(g - want).max() <= 5e-4 * np.abs(want).max()


def test_two_contexts_on_two_streams_concurrently(dev):
    # contexts are independent: two analyses enqueued on two streams at once give the same
    # bits as the same analyses run one after the other
    probs = _problems(4000)[:2]
    ins = []
    for p in probs:
        X = torch.from_numpy(p["X"]).to(dev)
        idx = torch.from_numpy(p["idx"]).to(dev)
        y = torch.from_numpy(p["y"]).to(dev)
        ins.append((X, idx, y, p))
    seq = []
    for X, idx, y, p in ins:
        post = torch.empty((p["M"], X.shape[1]), device=dev)
        with ensf.Context(precision="fp32") as ctx:
            ensf.ensf_analysis(ctx.handle, X, post, idx, y, p["sig"], p["K"], p["seed"], p["fid"])
            assert ensf.ensf_sync_status(ctx.handle)[0] == ensf.ENSF_OK
        seq.append(post.cpu().numpy())
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    for s in streams:
        s.wait_stream(torch.cuda.current_stream())
    ctxs = [ensf.Context(precision="fp32"), ensf.Context(precision="fp32")]
    outs = []
    try:
        for (X, idx, y, p), s, c in zip(ins, streams, ctxs):
            post = torch.empty((p["M"], X.shape[1]), device=dev)
            ensf.ensf_analysis(c.handle, X, post, idx, y, p["sig"], p["K"], p["seed"], p["fid"],
                               stream=s)
            outs.append(post)
        for c in ctxs:
            assert ensf.ensf_sync_status(c.handle)[0] == ensf.ENSF_OK
    finally:
        for c in ctxs:
            c.destroy()
    for a, b in zip(seq, outs):
        np.testing.assert_array_equal(a, b.cpu().numpy())
