"""Assimilation cycle on the GPU (reduced size): truth and physics forecast by the SQG
model, learned forecast by the trained conv surrogate or a ViT surrogate, split-BF16 EnSF
analysis.

Checks: the cycle stays finite and bounded; at the observed components the analysis
error is below the forecast error every cycle; the trained network is a useful forecast
model (validation error well below persistence, its cycled analysis beats carrying the
analysis over without a forecast model, and its mean analysis RMSE stays within
CONV_VS_SPECTRAL of the spectral forecast's).  In this twin setting the physics forecast is the
truth's own model, so the network's expected gain over it is speed (reported).
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2407_12168_amd import cycle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


# bar on the mean analysis RMSE of the learned-forecast cycle relative to the spectral one
CONV_VS_SPECTRAL = 1.5

CFG = cycle.CycleConfig(grid=64, members=64, cycles=6, pseudo_steps=400, sqg_dt=0.025,
                        steps_per_cycle=10, spinup_steps=800)


def test_cycle_with_physics_forecast(dev):
    res = cycle.run_cycle(CFG, "sqg", dev=dev, log=print)
    assert all(np.isfinite(res.rmse)) and max(res.rmse) < 3.0
    assert all(a < f for a, f in zip(res.rmse_obs, res.rmse_forecast_obs))


def test_trained_surrogate_beats_no_forecast_and_tracks_physics(dev):
    x, y = cycle.training_pairs(768, CFG, dev)
    xv, yv = cycle.training_pairs(64, CFG, dev, seed=99, perturbed=0.0)
    base = float(torch.mean((xv - yv) ** 2))
    sur, hist = cycle.train_surrogate(x, y, epochs=20, batch=32, lr=1e-3, val=(xv, yv), log=print)
    print(f"validation mse: persistence {base:.4e}, surrogate {hist[-1]['val_mse']:.4e}")
    assert hist[-1]["val_mse"] < 0.7 * base
    conv = cycle.run_cycle(CFG, "conv", surrogate=sur, dev=dev)
    pers = cycle.run_cycle(CFG, "persistence", dev=dev)
    phys = cycle.run_cycle(CFG, "sqg", dev=dev)
    sur.destroy()
    m = lambda r: float(np.mean(r.rmse[1:]))
    f = lambda r: float(np.mean(r.rmse_forecast[1:]))
    print(f"mean rmse (cycles 1+) analysis / forecast: conv {m(conv):.4f} / {f(conv):.4f}, "
          f"persistence {m(pers):.4f} / {f(pers):.4f}, sqg {m(phys):.4f} / {f(phys):.4f}; "
          f"forecast ms conv {1e3 * np.mean(conv.forecast_s):.2f}, "
          f"sqg {1e3 * np.mean(phys.forecast_s):.2f}")
    assert f(conv) < f(pers)
    # the spectral forecast is the truth's own model in this twin experiment, so the learned
    # forecast cannot beat it on accuracy; it must keep the analysis within a factor of it
    # (the full-size cycle measures 0.88x: the network forecast is also smoother)
    assert m(conv) < CONV_VS_SPECTRAL * m(phys)


# a reduced ViT (the Table II architecture with 4 layers of width 256) keeps the test short;
# the Table II model itself runs in `bench.py --vit-cycle`
VIT_ARCH = dict(patch=4, layers=4, heads=4, embed=256, mlp_hidden=1024)
VIT_CFG = cycle.CycleConfig(grid=64, members=64, cycles=12, pseudo_steps=400, sqg_dt=0.025,
                            steps_per_cycle=10, spinup_steps=800)


def test_vit_forecast_cycle_and_online_training(dev):
    """The ViT surrogate, trained on SQG pairs by the library's kernels, is a usable forecast
    model (better than persistence on validation pairs and in the cycle), and online training
    on the observations (OnlineTuning) keeps the cycle finite and bounded."""
    x, y = cycle.training_pairs(1024, VIT_CFG, dev)
    xv, yv = cycle.training_pairs(64, VIT_CFG, dev, seed=99, perturbed=0.0)
    base = float(torch.mean((xv - yv) ** 2))
    net, hist = cycle.train_vit(x, y, epochs=20, batch=32, lr=3e-4, val=(xv, yv), **VIT_ARCH)
    print(f"validation mse: persistence {base:.4e}, ViT {hist[-1]['val_mse']:.4e}")
    assert hist[-1]["val_mse"] < base
    f = lambda r: float(np.mean(r.rmse_forecast[2:]))
    vitr = cycle.run_cycle(VIT_CFG, "vit", surrogate=net, dev=dev)
    pers = cycle.run_cycle(VIT_CFG, "persistence", dev=dev)
    onl = cycle.run_cycle(VIT_CFG, "vit", surrogate=net, dev=dev,
                          online=cycle.OnlineTuning(steps=2, lr=3e-6, window=4))
    net.destroy()
    print(f"mean forecast rmse (cycles 2+): ViT {f(vitr):.4f}, online {f(onl):.4f}, "
          f"persistence {f(pers):.4f}")
    assert f(vitr) < f(pers)
    assert all(np.isfinite(onl.rmse)) and max(onl.rmse) < 3.0
