"""Host logic of bench.py (CPU): the one-GPU limit and the roofline arithmetic."""
import importlib.util
import os
import subprocess
import sys
from types import SimpleNamespace

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_roofline_prices_the_dominant_kernel():
    b = _bench()
    p = SimpleNamespace(n_members=256, dim=32768)
    flops = 2.0 * 256 * 256 * 32768
    # W.X dominant: achieved = flops / its launch time, against the FP32 MFMA peak
    r = b.roofline([p], "fp32", [0.043, 0.009, 0.050], config=2)
    assert r["kernel"] == "k_wx" and r["bound"] == "mfma" and r["unit"] == "TFLOP/s"
    assert r["achieved"] == pytest.approx(flops / 0.050e-3 / 1e12, rel=1e-3)
    assert r["frac"] == pytest.approx(r["achieved"] / 157.3, rel=1e-3)
    assert r["traffic"] == b.MEASURED_TRAFFIC[(2, "fp32", "k_wx")]
    # Gram dominant, and no measured traffic for it: null
    r = b.roofline([p], "bf16x3", [0.060, 0.009, 0.050], config=2)
    assert r["kernel"] == "k_gram" and r["peak"] == 2500.0 and r["traffic"] is None
    # the degenerate-weight W.X is not priced as a contraction: the Gram is
    r = b.roofline([p], "fp32", [0.043, 0.009, 0.050], config=2, wx_sparse=True)
    assert r["kernel"] == "k_gram" and r["traffic"] is None
    # batched: flops add over the filters
    q = SimpleNamespace(n_members=64, dim=8192)
    r = b.roofline([p, q], "fp32", [0.010, 0.001, 0.020], config=4)
    want = (flops + 2.0 * 64 * 64 * 8192) / 0.020e-3 / 1e12
    assert r["achieved"] == pytest.approx(want, rel=1e-3) and r["traffic"] is None


def test_cycle_rejects_online_training_without_a_learned_forecast():
    from paper_2407_12168_amd import cycle
    cfg = cycle.CycleConfig(grid=32, members=8, cycles=1)
    with pytest.raises(ValueError):
        cycle.run_cycle(cfg, "sqg", online=cycle.OnlineTuning())
    with pytest.raises(ValueError):
        cycle.run_cycle(cfg, "persistence", online=cycle.OnlineTuning())
    with pytest.raises(ValueError):
        cycle.run_cycle(cycle.CycleConfig(obs_op="arctan"), "conv", surrogate=object(),
                        online=cycle.OnlineTuning())
    with pytest.raises(ValueError):
        cycle.run_cycle(cfg, "spectral")
    with pytest.raises(ValueError):
        cycle.run_cycle(cfg, "vit")
