"""GPU test of ensf_analysis_noalloc (the entry point that allocates nothing and runs in the
library's static scratch buffer), through the C ABI.

Two calls in a row, the second on a smaller problem (the scratch keeps the first call's
contents, so this also checks that everything that must start at zero is cleared), each
compared bit for bit with ensf_analysis on a context without a tune table (the same tiles,
so the same arithmetic), plus: both precisions, the implicit step, the counters output,
device memory unchanged across a call, and the synchronous rejection of a problem larger
than the scratch buffer.  The oracle comparison of the same analysis is in the parity tests
of ensf_analysis."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import workloads
from oracle import ensf as O
from paper_2407_12168_amd import ensf

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _inputs(dev, p):
    X = torch.from_numpy(p.X).to(dev)
    idx = torch.from_numpy(p.obs_idx).to(dev)
    val = torch.from_numpy(p.obs_val).to(dev)
    return X, idx, val


def _with_context(dev, p, n_particles, **opts):
    X, idx, val = _inputs(dev, p)
    post = torch.empty((n_particles, p.dim), device=dev)
    with ensf.Context(tune_cache=None, **opts) as ctx:
        ensf.ensf_analysis(ctx.handle, X, post, idx, val, p.sigma_o, p.n_steps, p.seed,
                           p.filter_id)
        st, bad = ensf.ensf_sync_status(ctx.handle)
    assert st == ensf.ENSF_OK, (st, bad)
    return post.cpu()


def _noalloc(dev, p, n_particles, counters=None, **opts):
    X, idx, val = _inputs(dev, p)
    post = torch.full((n_particles, p.dim), float("nan"), device=dev)
    torch.cuda.synchronize()
    ensf.ensf_analysis_noalloc(X, post, idx, val, p.sigma_o, p.n_steps, p.seed, p.filter_id,
                               counters=counters, **opts)
    torch.cuda.synchronize()
    return post.cpu()


@pytest.mark.parametrize("precision,lik_step", [("fp32", "explicit"), ("bf16x3", "implicit")])
def test_noalloc_matches_ensf_analysis_two_calls(dev, precision, lik_step):
    big = workloads.make_problem(2, 40, 48, 70, 0.05, 24, data_seed=11, seed=12, obs_fraction=0.3)
    # K >= 1 / sigma_o^2 for the small one: the explicit step is then contracting and its
    # trajectory comparable with the oracle's
    small = workloads.make_problem(2, 16, 24, 33, 0.2, 30, data_seed=13, seed=14, filter_id=3)
    opts = dict(precision=precision, lik_step=lik_step)
    counters = torch.zeros(2, dtype=torch.int64, device=dev)
    got_big = _noalloc(dev, big, 70, counters, **opts)
    got_small = _noalloc(dev, small, 29, counters, **opts)
    want_big = _with_context(dev, big, 70, **opts)
    want_small = _with_context(dev, small, 29, **opts)
    print(f"{precision}: big max|diff| {float((got_big - want_big).abs().max()):.3e}, "
          f"small {float((got_small - want_small).abs().max()):.3e}")
    assert torch.equal(got_big, want_big)
    assert torch.equal(got_small, want_small)
    assert counters.cpu().tolist() == [0, 0]
    # and the small problem against the FP64 oracle at the filter's bar (particle subset)
    rows = [0, 28]
    ref = O.analysis(small.X, small.obs_idx, small.obs_val, small.sigma_o, small.n_steps,
                     small.seed, filter_id=small.filter_id, particle_ids=rows,
                     lik_step=lik_step)
    got = got_small.numpy().astype(np.float64)[rows]
    assert O.rel_l2(got, ref) < 1e-3


def test_noalloc_allocates_nothing_and_reports_counters(dev):
    p = workloads.make_problem(2, 32, 32, 40, 0.05, 10, data_seed=21, seed=22)
    X, idx, val = _inputs(dev, p)
    post = torch.empty((40, p.dim), device=dev)
    counters = torch.zeros(2, dtype=torch.int64, device=dev)
    # invalid observations are skipped and counted in counters[1]
    bad_idx = idx.clone()
    bad_idx[:3] = p.dim + 5
    ensf.ensf_analysis_noalloc(X, post, bad_idx, val, p.sigma_o, p.n_steps, p.seed,
                               counters=counters)
    torch.cuda.synchronize()
    assert counters.cpu().tolist() == [0, 3]
    free0, _ = torch.cuda.mem_get_info()
    ensf.ensf_analysis_noalloc(X, post, idx, val, p.sigma_o, p.n_steps, p.seed,
                               counters=counters)
    torch.cuda.synchronize()
    free1, _ = torch.cuda.mem_get_info()
    assert free1 == free0, (free0, free1)
    assert counters.cpu().tolist() == [0, 3]


def test_noalloc_rejects_problems_beyond_the_scratch(dev):
    # 256 members x 65536 components: the FP32 prior copy alone is 64 MiB
    N, d = 256, 65536
    X = torch.zeros((N, d), device=dev)
    post = torch.empty((N, d), device=dev)
    with pytest.raises(ensf.EnsfError) as e:
        ensf.ensf_analysis_noalloc(X, post, None, None, 0.05, 5, 1)
    assert e.value.status == ensf.ENSF_ESCRATCH
    with pytest.raises(ensf.EnsfError) as e:
        ensf.ensf_analysis_noalloc(X[:4], post[:4], None, None, 0.05, 0, 1)
    assert e.value.status == ensf.ENSF_EINVAL
