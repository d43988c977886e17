"""Pins of the FP64 SQG stepper: textbook Eady growth rate of a small single mode,
conservation of temperature variance in the inviscid no-shear limit, and 4th-order
convergence of the RK4 time stepping."""
import numpy as np
import pytest

import workloads
from oracle.sqg import SQG, eady_growth_rate


@pytest.mark.parametrize("m", [3, 5, 7])
def test_linear_eady_growth_rate(m):
    n, lx = 32, 20.0
    model = SQG(n=n, lx=lx, dt=0.05, diff_efold=np.inf)
    k = 2 * np.pi * m / lx
    x = np.arange(n) * lx / n
    rng = np.random.default_rng(m)
    ph = rng.uniform(0, 2 * np.pi, 2)
    theta = 1e-9 * np.stack([np.cos(k * x + ph[0]), 0.7 * np.cos(k * x + ph[1])])
    theta = np.broadcast_to(theta[:, None, :], (2, n, n)).copy()
    th = model.fft(theta) * model.mask
    amps = []
    for step in range(600):
        th = model.step_spectral(th)
        if step % 100 == 99:
            amps.append(np.abs(th[:, 0, m]).sum())
    rate = np.log(amps[-1] / amps[-2]) / (100 * model.dt)
    want = eady_growth_rate(k, k)
    assert want > 0.05
    assert abs(rate - want) <= 0.01 * want


def test_short_waves_beyond_cutoff_do_not_grow():
    n, lx, m = 32, 20.0, 9                   # K = 2.83 > 2.4 (Eady short-wave cutoff)
    model = SQG(n=n, lx=lx, dt=0.05, diff_efold=np.inf)
    k = 2 * np.pi * m / lx
    assert eady_growth_rate(k, k) == 0.0
    x = np.arange(n) * lx / n
    theta = 1e-9 * np.stack([np.cos(k * x), 0.5 * np.sin(k * x)])
    theta = np.broadcast_to(theta[:, None, :], (2, n, n)).copy()
    th0 = model.fft(theta) * model.mask
    th = th0
    for _ in range(400):
        th = model.step_spectral(th)
    assert np.abs(th[:, 0, m]).sum() < 3 * np.abs(th0[:, 0, m]).sum()


def test_variance_conserved_without_shear_and_diffusion():
    model = SQG(n=32, lx=20.0, shear=0.0, dt=0.01, diff_efold=np.inf)
    theta = workloads.smooth_fields(np.random.default_rng(1), 2, 32, 32, slope=4.0) * 0.3
    th = model.fft(theta) * model.mask
    v0 = np.sum(model.ifft(th) ** 2, axis=(-2, -1))
    for _ in range(50):
        th = model.step_spectral(th)
    v1 = np.sum(model.ifft(th) ** 2, axis=(-2, -1))
    np.testing.assert_allclose(v1, v0, rtol=50 * 1e-10)


def test_rk4_fourth_order_in_time():
    rng = np.random.default_rng(2)
    theta = workloads.smooth_fields(rng, 2, 32, 32, slope=4.0) * 0.5
    T = 0.4
    ref = SQG(n=32, dt=T / 256, diff_efold=np.inf).run(theta, 256)
    errs = []
    for nst in (8, 16, 32):
        out = SQG(n=32, dt=T / nst, diff_efold=np.inf).run(theta, nst)
        errs.append(np.abs(out - ref).max())
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 13.0 < r1 < 19.0 and 13.0 < r2 < 19.0, errs
