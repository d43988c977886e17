"""Pins of the FP64 conv-surrogate oracle: forward vs a library correlation with wrap
boundary, gradients vs central finite differences, Adam vs its closed form on step 1."""
import numpy as np
import pytest
from scipy import signal

from oracle import conv


def test_conv_forward_matches_scipy_wrap_correlation():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((2, 3, 8, 8))
    w = rng.standard_normal((4, 3, 3, 3))
    b = rng.standard_normal(4)
    out = conv.conv3x3(x, w, b)
    for n in range(2):
        for o in range(4):
            ref = b[o] + sum(signal.correlate2d(x[n, c], w[o, c], mode="same", boundary="wrap")
                             for c in range(3))
            np.testing.assert_allclose(out[n, o], ref, rtol=1e-12, atol=1e-12)


def test_parameter_count_and_flops_of_the_surrogate():
    params = conv.init_params(np.random.default_rng(1))
    assert conv.n_params(params) == 150082
    assert conv.forward_flops(128, 128) == pytest.approx(4.91e9, rel=1e-3)


def test_gradients_match_finite_differences():
    rng = np.random.default_rng(2)
    params = conv.init_params(rng, c0=2, width=4, layers=3)
    params = [(w * 3.0, rng.standard_normal(b.shape) * 0.1) for w, b in params]
    x = rng.standard_normal((2, 2, 8, 8))
    target = rng.standard_normal((2, 2, 8, 8))
    _, grads = conv.loss_and_grads(params, x, target)
    h = 1e-6
    for i in range(len(params)):
        for j in (0, 1):
            arr = params[i][j]
            flat_idx = rng.choice(arr.size, size=min(6, arr.size), replace=False)
            for fi in flat_idx:
                idx = np.unravel_index(fi, arr.shape)
                orig = arr[idx]
                arr[idx] = orig + h
                lp = conv.mse(conv.forward(params, x), target)
                arr[idx] = orig - h
                lm = conv.mse(conv.forward(params, x), target)
                arr[idx] = orig
                fd = (lp - lm) / (2 * h)
                assert abs(grads[i][j][idx] - fd) <= 1e-7 * max(1.0, abs(fd)), (i, j, idx)


def test_input_gradient_matches_finite_differences():
    rng = np.random.default_rng(3)
    x = rng.standard_normal((1, 3, 6, 6))
    w = rng.standard_normal((2, 3, 3, 3))
    g = rng.standard_normal((1, 2, 6, 6))
    gx, _, _ = conv.conv3x3_backward(x, w, g)
    h = 1e-6
    for idx in [(0, 0, 0, 0), (0, 2, 5, 1), (0, 1, 3, 5)]:
        xp, xm = x.copy(), x.copy()
        xp[idx] += h
        xm[idx] -= h
        fd = (np.sum(g * conv.conv3x3(xp, w, np.zeros(2)))
              - np.sum(g * conv.conv3x3(xm, w, np.zeros(2)))) / (2 * h)
        assert abs(gx[idx] - fd) < 1e-7


def test_gelu_and_derivative():
    u = np.array([-3.0, -0.5, 0.0, 0.7, 2.0])
    np.testing.assert_allclose(conv.gelu(np.array([0.0])), [0.0])
    h = 1e-6
    np.testing.assert_allclose(conv.gelu_grad(u), (conv.gelu(u + h) - conv.gelu(u - h)) / (2 * h),
                               rtol=1e-8)
    # large positive inputs pass through, large negative ones vanish
    np.testing.assert_allclose(conv.gelu(np.array([10.0, -10.0])), [10.0, 0.0], atol=1e-12)


def test_adam_first_step_is_signed_learning_rate():
    rng = np.random.default_rng(4)
    params = [(rng.standard_normal((2, 1, 3, 3)), rng.standard_normal(2))]
    grads = [(rng.standard_normal((2, 1, 3, 3)), rng.standard_normal(2))]
    state = [[(np.zeros_like(p), np.zeros_like(p)) for p in params[0]]]
    new = conv.adam_step(params, grads, state, lr=1e-3, step=1)
    # bias-corrected first step: p - lr * g / (|g| + eps)
    for (p, g, q) in zip(params[0], grads[0], new[0]):
        np.testing.assert_allclose(q, p - 1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-12)
