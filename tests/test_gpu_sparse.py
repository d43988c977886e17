"""Degenerate-weight W.X (ensf_options.wx_sparse): tiles whose particle rows have at most 8
weights >= 2^-30 gather xhat from those members instead of the dense product.  The dropped
weights are below FP32 resolution of a unit-sum row, so the result must meet the same bar
against the FP64 oracle (which always uses every member) as the dense path: rel-L2 <= 1e-3 of
whole trajectories at EM-stable K, and at the literal K with the implicit step.  Early
pseudo-steps (near-uniform weights) run the dense tiles of the same kernel, later ones the
gathers, so both branches are exercised."""
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


def _run(dev, p, precision, sparse=True, lik_step="explicit", n_particles=None):
    X = torch.from_numpy(np.ascontiguousarray(p.X)).to(dev)
    post = torch.empty((n_particles or p.n_members, p.dim), device=dev)
    idx = torch.from_numpy(p.obs_idx).to(dev)
    val = torch.from_numpy(p.obs_val).to(dev)
    with ensf.Context(precision=precision, obs_op=p.obs_op, lik_step=lik_step,
                      wx_sparse=sparse) as ctx:
        ensf.ensf_analysis(ctx.handle, X, post, idx, val, p.sigma_o, p.n_steps, p.seed,
                           p.filter_id)
        st, nbad = ensf.ensf_sync_status(ctx.handle)
    assert st == ensf.ENSF_OK, (st, nbad)
    return post.cpu().numpy().astype(np.float64)


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_sparse_config1_stable_k_full_trajectory(dev, precision):
    p = workloads.config_problem(1, n_steps=400)
    want = O.analysis(p.X, p.obs_idx, p.obs_val, p.sigma_o, p.n_steps, p.seed)
    got = _run(dev, p, precision)
    err = O.rel_l2(got, want)
    print(f"c1 K=400 sparse {precision}: particles rel-L2 {err:.2e}")
    assert err <= 1e-3


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_sparse_config2_stable_k_particle_subset(dev, precision):
    p = workloads.config_problem(2, n_steps=400)
    got = _run(dev, p, precision)
    rows = [0, 200]
    want = O.analysis(p.X, p.obs_idx, p.obs_val, p.sigma_o, p.n_steps, p.seed,
                      particle_ids=rows)
    err = O.rel_l2(got[rows], want)
    dense = _run(dev, p, precision, sparse=False)
    dd = O.rel_l2(got, dense)
    print(f"c2 K=400 sparse {precision}: particles {rows} rel-L2 {err:.2e}; vs dense {dd:.2e}")
    assert err <= 1e-3 and dd <= 1e-4


def test_sparse_literal_k_implicit_config2(dev):
    p = workloads.config_problem(2)
    got = _run(dev, p, "bf16x3", lik_step="implicit")
    rows = [5, 250]
    want = O.analysis(p.X, p.obs_idx, p.obs_val, p.sigma_o, p.n_steps, p.seed,
                      particle_ids=rows, lik_step="implicit")
    err = O.rel_l2(got[rows], want)
    print(f"c2 K=100 implicit sparse bf16x3: rel-L2 {err:.2e}")
    assert err <= 1e-3


def test_sparse_ragged_and_batched(dev):
    # ragged sizes (d not a multiple of 4, M_p != N) through the batched call
    specs = [(9, 1001, 13, 60, 0.5), (40, 2050, 33, 50, 0.5), (70, 515, 70, 40, 0.6)]
    tens, descs, probs = [], [], []
    for f, (N, d, M, K, sig) in enumerate(specs):
        rng = np.random.default_rng(900 + f)
        X = rng.standard_normal((N, d)).astype(np.float32)
        idx = np.sort(rng.choice(d, d // 2, replace=False)).astype(np.int32)
        y = np.arctan(rng.standard_normal(idx.size)).astype(np.float32)
        Xg = torch.from_numpy(X).to(dev)
        post = torch.empty((M, d), device=dev)
        ig = torch.from_numpy(idx).to(dev)
        yg = torch.from_numpy(y).to(dev)
        tens.append((Xg, post, ig, yg))
        descs.append(ensf.make_problem(Xg, post, ig, yg, sig, K, 31 + f, f))
        probs.append((X, idx, y, sig, K, 31 + f, f, M))
    with ensf.Context(precision="fp32", wx_sparse=True) as ctx:
        ensf.ensf_analysis_batched(ctx.handle, descs)
        st, nbad = ensf.ensf_sync_status(ctx.handle)
    assert st == ensf.ENSF_OK, (st, nbad)
    for (X, idx, y, sig, K, seed, f, M), t in zip(probs, tens):
        want = O.analysis(X, idx, y, sig, K, seed, filter_id=f, n_particles=M)
        got = t[1].cpu().numpy().astype(np.float64)
        err = np.abs(got - want).max() / np.abs(want).max()
        print(f"sparse batched filter {f}: max rel diff {err:.2e}")
        assert err <= 5e-4
