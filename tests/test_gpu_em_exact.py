"""GPU form of the exact Euler-Maruyama pin (eq. 7): one forecast member, so the
Monte-Carlo prior score of eq. 15 is the exact score of N(alpha x, beta^2) and every
particle component is exactly Gaussian with the closed-form mean and variance of the
discrete recursion (`oracle.linear_gaussian`).  Half the components are observed through
the identity operator; each group pools n_particles x d/2 i.i.d. components and must match
the recursion within 4 standard errors (mean) and the chi-square band (variance), with no
additive allowance.  FP32 rounding of the scheme is below 1e-3 of a standard error here."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import linear_gaussian as lg
from paper_2407_12168_amd import ensf

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
@pytest.mark.parametrize("lik_step,sigma_o,K", [("explicit", 0.3, 100), ("implicit", 0.05, 100),
                                                ("explicit", 0.5, 37)])
def test_one_member_statistics_equal_recursion(dev, precision, lik_step, sigma_o, K):
    mu, y, d, P = 1.0, -1.0, 32768, 64
    X = torch.full((1, d), mu, device=dev)
    post = torch.empty((P, d), device=dev)
    idx = torch.arange(0, d, 2, dtype=torch.int32, device=dev)
    val = torch.full((d // 2,), y, device=dev)
    with ensf.Context(precision=precision, obs_op="linear", lik_step=lik_step) as ctx:
        ensf.ensf_analysis(ctx.handle, X, post, idx, val, sigma_o, K, 4242 + K)
        st, nbad = ensf.ensf_sync_status(ctx.handle)
    assert st == ensf.ENSF_OK, (st, nbad)
    Z = post.cpu().numpy().astype(np.float64)
    for group, (A, B) in ((Z[:, 0::2], (y / sigma_o ** 2, 1.0 / sigma_o ** 2)),
                          (Z[:, 1::2], (0.0, 0.0))):
        m, v = lg.em_recursion(mu, 0.0, A, B, K, lik_step=lik_step)
        n = group.size
        zm = (group.mean() - m) / np.sqrt(v / n)
        zv = (group.var(ddof=1) / v - 1.0) / np.sqrt(2.0 / (n - 1))
        print(f"{precision} {lik_step} sigma_o={sigma_o} K={K}: mean z {zm:+.2f}, var z {zv:+.2f}")
        assert abs(zm) < 4.0 and abs(zv) < 4.0
