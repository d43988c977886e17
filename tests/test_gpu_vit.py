"""GPU parity of the ViT forecast surrogate (include/ensf_vit.h) against the FP64 oracle
(oracle/vit.py) at a reduced configuration that still has every piece of the Table II model
(2 x 32 x 32 states, patch 4 -> 64 tokens of 32 values, 2 layers, 2 heads of 32, embed 64,
MLP 128, batch 2): forward output, loss, every parameter tensor's gradient, one Adam step;
then the Table II 64^2 configuration itself (157M-class, 12 layers, embed 1024) for a few
training steps (finite, decreasing loss on a fixed batch).

Tolerances: the products take BF16 operands (relative rounding 2^-9 per operand, FP32
accumulation), so per-tensor relative L2 errors of a few 1e-3 are expected; the bars are
2e-2 for the forward output (net part), the loss and the gradients, and 5e-2 for the few
gradient tensors that are a single small reduction (LayerNorm gains and biases, positions),
whose relative error is that of a short sum of rounded terms.  Adam is checked against the
oracle's Adam applied to the GPU's own gradient (FP32 arithmetic against FP64: 1e-5)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import vit as V
from paper_2407_12168_amd import vit

pytestmark = pytest.mark.gpu

CFG = V.Config(channels=2, height=32, width=32, patch=4, layers=2, heads=2, embed=64,
               mlp_hidden=128)
BATCH = 2


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _model(cfg, max_batch, seed=0):
    return vit.ViT(channels=cfg.channels, height=cfg.height, width=cfg.width, patch=cfg.patch,
                   layers=cfg.layers, heads=cfg.heads, embed=cfg.embed,
                   mlp_hidden=cfg.mlp_hidden, max_batch=max_batch, seed=seed)


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30))


@pytest.fixture(scope="module")
def case():
    rng = np.random.default_rng(17)
    flat = V.init_params(CFG, rng)
    flat += 0.05 * rng.standard_normal(flat.size)           # away from the symmetric init
    flat = flat.astype(np.float32)
    x = rng.standard_normal((BATCH, 2, 32, 32)).astype(np.float32)
    target = (x + 0.3 * rng.standard_normal(x.shape)).astype(np.float32)
    f64 = flat.astype(np.float64)
    y_ref, _ = V.forward(CFG, f64, x.astype(np.float64))
    loss_ref, g_ref = V.loss_and_grad(CFG, f64, x.astype(np.float64), target.astype(np.float64))
    return flat, x, target, y_ref, loss_ref, g_ref


def test_param_count_matches_oracle(dev):
    with _model(CFG, BATCH) as m:
        assert vit.ensf_vit_num_params(m.handle) == V.num_params(CFG)
    with _model(V.TABLE2_64, 1) as m:
        assert vit.ensf_vit_num_params(m.handle) == V.num_params(V.TABLE2_64) == 151485472


def test_forward_loss_and_every_gradient_match_oracle(dev, case):
    flat, x, target, y_ref, loss_ref, g_ref = case
    xg = torch.from_numpy(x).to(dev)
    tg = torch.from_numpy(target).to(dev)
    with _model(CFG, BATCH) as m:
        vit.ensf_vit_set_params(m.handle, flat)
        y = torch.empty_like(xg)
        vit.ensf_vit_forward(m.handle, xg, y)
        grad = torch.empty(flat.size, device=dev)
        loss = vit.ensf_vit_grad(m.handle, xg, tg, grad)
        torch.cuda.synchronize()
        y = y.cpu().numpy().astype(np.float64)
        g = grad.cpu().numpy().astype(np.float64)
    net_err = _rel(y - x, y_ref - x)
    print(f"forward net part rel-L2 {net_err:.2e}; loss {loss:.6f} vs {loss_ref:.6f}")
    assert net_err < 2e-2
    assert abs(loss - loss_ref) / loss_ref < 2e-2
    o = 0
    worst = {}
    for name, shape in V.param_shapes(CFG):
        n = int(np.prod(shape))
        err = _rel(g[o:o + n], g_ref[o:o + n])
        worst[name] = err
        tol = 5e-2 if name.startswith(("ln", "b_", "pos")) else 2e-2
        assert err < tol, (name, err)
        o += n
    print("gradient rel-L2 per tensor: " +
          ", ".join(f"{k} {v:.1e}" for k, v in sorted(worst.items(), key=lambda kv: -kv[1])[:6]))


@pytest.mark.parametrize("size,batch", [(64, 1), (128, 2)])
def test_one_layer_at_table2_widths_matches_oracle(dev, size, batch):
    """One transformer layer at the Table II widths: 64^2 (embed 1024, 8 heads, MLP 4096, 256
    tokens per state) and 128^2 (embed 2048, 8 heads, MLP 8192, 1024 tokens).  The products
    here use the large tiles (k-step 64, one and two LDS stages) that the reduced
    configuration's short contractions never reach; 128^2 also runs the widest LayerNorm and
    the 1024-token attention rows and, at batch 2 (2048 tokens), the 256 x 128 tiles: the
    MLP's 2048 x 8192 products with contraction 2048 (the forward of the first linear map,
    the input gradient of the second) fill two of them per compute unit."""
    D = 1024 if size == 64 else 2048
    cfg = V.Config(channels=2, height=size, width=size, patch=4, layers=1, heads=8, embed=D,
                   mlp_hidden=4 * D)
    rng = np.random.default_rng(23)
    flat = V.init_params(cfg, rng)
    flat += 0.02 * rng.standard_normal(flat.size)
    flat = flat.astype(np.float32)
    x = rng.standard_normal((batch, 2, size, size)).astype(np.float32)
    target = (x + 0.3 * rng.standard_normal(x.shape)).astype(np.float32)
    f64 = flat.astype(np.float64)
    loss_ref, g_ref = V.loss_and_grad(cfg, f64, x.astype(np.float64), target.astype(np.float64))
    xg = torch.from_numpy(x).to(dev)
    tg = torch.from_numpy(target).to(dev)
    with _model(cfg, batch) as m:
        vit.ensf_vit_set_params(m.handle, flat)
        grad = torch.empty(flat.size, device=dev)
        loss = vit.ensf_vit_grad(m.handle, xg, tg, grad)
        torch.cuda.synchronize()
        g = grad.cpu().numpy().astype(np.float64)
    assert abs(loss - loss_ref) / loss_ref < 2e-2
    o = 0
    worst = {}
    for name, shape in V.param_shapes(cfg):
        n = int(np.prod(shape))
        err = _rel(g[o:o + n], g_ref[o:o + n])
        worst[name] = err
        tol = 5e-2 if name.startswith(("ln", "b_", "pos")) else 2e-2
        assert err < tol, (name, err)
        o += n
    print(f"Table II {size}^2 widths, batch {batch}, gradient rel-L2 per tensor: " +
          ", ".join(f"{k} {v:.1e}" for k, v in sorted(worst.items(), key=lambda kv: -kv[1])[:6]))


def test_adam_step_matches_oracle_adam_on_the_gpu_gradient(dev, case):
    flat, x, target, *_ = case
    xg = torch.from_numpy(x).to(dev)
    tg = torch.from_numpy(target).to(dev)
    lr = 1e-3
    with _model(CFG, BATCH) as m:
        vit.ensf_vit_set_params(m.handle, flat)
        grad = torch.empty(flat.size, device=dev)
        vit.ensf_vit_grad(m.handle, xg, tg, grad)
        g = grad.cpu().numpy().astype(np.float64)
        vit.ensf_vit_train_step(m.handle, xg, tg, lr)
        got = vit.ensf_vit_get_params(m.handle).astype(np.float64)
    want, _, _ = V.adam(flat.astype(np.float64), g, np.zeros_like(g), np.zeros_like(g), 1, lr)
    step_got, step_want = got - flat, want - flat
    assert _rel(step_got, step_want) < 1e-5


@pytest.mark.parametrize("mlp_hidden", [128, 96])
def test_optimizer_bf16_copies_equal_fresh_copies(dev, mlp_hidden):
    # the optimizer step rewrites the BF16 weight copies (row-major and transposed) itself;
    # they must equal the copies made from the FP32 weights it wrote (96: matrices that end
    # in part-tiles of the optimizer's 64 x 64 tiles, as the 32-wide patch and head do)
    cfg = V.Config(channels=2, height=32, width=32, patch=4, layers=2, heads=2, embed=64,
                   mlp_hidden=mlp_hidden)
    g = torch.Generator(device="cpu").manual_seed(11)
    x = torch.randn((BATCH, 2, 32, 32), generator=g).to(dev)
    t = (x + 0.3 * torch.randn(x.shape, generator=g).to(dev)).contiguous()
    with _model(cfg, BATCH, seed=2) as m:
        n = vit.ensf_vit_num_params(m.handle)
        for _ in range(3):
            vit.ensf_vit_train_step(m.handle, x, t, 1e-3)
        y1, g1 = torch.empty_like(x), torch.empty(n, device=dev)
        vit.ensf_vit_forward(m.handle, x, y1)
        vit.ensf_vit_grad(m.handle, x, t, g1)
        vit.ensf_vit_set_params(m.handle, vit.ensf_vit_get_params(m.handle))
        y2, g2 = torch.empty_like(x), torch.empty(n, device=dev)
        vit.ensf_vit_forward(m.handle, x, y2)
        vit.ensf_vit_grad(m.handle, x, t, g2)
    torch.cuda.synchronize()
    assert torch.equal(y1, y2)
    assert torch.equal(g1, g2)


def test_training_reduces_the_loss_at_the_reduced_and_table2_sizes(dev):
    # a learnable map: the increment is a third of the shift by one grid column
    for cfg, batch, steps, lr in ((CFG, BATCH, 30, 1e-4), (V.TABLE2_64, 2, 6, 2e-5)):
        g = torch.Generator(device="cpu").manual_seed(3)
        x = torch.randn((batch, cfg.channels, cfg.height, cfg.width), generator=g).to(dev)
        t = (x + 0.3 * (torch.roll(x, 1, dims=3) - x)).contiguous()
        with _model(cfg, batch, seed=5) as m:
            losses = [vit.ensf_vit_train_step(m.handle, x, t, lr) for _ in range(steps)]
        print(f"{cfg.embed}-wide, {cfg.layers} layers: loss {losses[0]:.4f} -> {losses[-1]:.4f}")
        assert all(np.isfinite(losses)) and losses[-1] < losses[0]
