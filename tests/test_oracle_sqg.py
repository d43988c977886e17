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


def test_thermal_relaxation_damps_every_mode_exactly():
    # with no flow (shear 0, no diffusion) a linear damping of rate 1/tau is exact per step
    model = SQG(n=16, lx=20.0, shear=0.0, dt=0.1, diff_efold=np.inf, relax_time=4.0)
    theta = 1e-12 * workloads.smooth_fields(np.random.default_rng(3), 2, 16, 16)
    out = model.run(theta, 10)
    kept = model.ifft(model.fft(theta) * model.mask)       # the model keeps 2/3 of the modes
    np.testing.assert_allclose(out, kept * np.exp(-1.0 / 4.0), rtol=1e-6, atol=1e-24)


def test_relaxed_turbulence_equilibrates():
    model = SQG(n=32, dt=0.025, relax_time=5.0)
    theta = workloads.smooth_fields(np.random.default_rng(4), 2, 32, 32)
    out = model.run(theta, 1200)
    assert np.all(np.isfinite(out)) and 0.2 < out.std() < 3.0


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
