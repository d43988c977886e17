"""GPU SQG model (FP64, hipFFT + own kernels) against the FP64 NumPy oracle: the same
equations, dealiasing, RK4 and hyperdiffusion, so results agree to round-off."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import workloads
from oracle.sqg import SQG
from paper_2407_12168_amd import sqg as G

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


@pytest.mark.parametrize("n,efold,tau", [(32, 0.25, 5.0), (64, np.inf, np.inf)])
def test_gpu_sqg_matches_oracle(dev, n, efold, tau):
    rng = np.random.default_rng(n)
    x = workloads.smooth_fields(rng, 6, n, n).reshape(3, 2, n, n)
    want = SQG(n=n, dt=0.025, diff_efold=efold, relax_time=tau).run(x, 20)
    with G.SQGModel(n=n, dt=0.025, diff_efold=efold, relax_time=tau, max_batch=2) as m:
        xg = torch.from_numpy(x).to(dev)
        yg = torch.empty_like(xg)
        m.run(xg, yg, 20)
        torch.cuda.synchronize()
        got = yg.cpu().numpy()
        y32 = torch.empty(x.shape, dtype=torch.float32, device=dev)
        m.run(xg.float().contiguous(), y32, 20)
        torch.cuda.synchronize()
    err = np.abs(got - want).max() / np.abs(want).max()
    err32 = np.abs(y32.cpu().numpy() - want).max() / np.abs(want).max()
    print(f"n={n}: FP64 max rel diff {err:.2e}, FP32 interface {err32:.2e}")
    assert err <= 1e-11
    assert err32 <= 1e-5
