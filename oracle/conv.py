"""FP64 oracle of the convolutional forecast surrogate (test infrastructure only).

Network: six 3x3 convolutions with periodic (circular) padding, channels
C0 -> 64 -> 64 -> 64 -> 64 -> 64 -> C0 (C0 = 2 levels), exact erf-GELU between layers,
residual output y = x + net(x); loss = mean squared error over all outputs; Adam
(Kingma & Ba, 2015) on FP32 master weights.  Training-FLOP accounting follows the
6 x tokens x parameters logic of eq. 18 (forward 2x, backward 4x).

Layout: NCHW arrays, weights (Cout, Cin, 3, 3), bias (Cout,).
"""
import math

import numpy as np
from scipy.special import erf


def _shift(a, dy, dx):
    """s[..., y, x] = a[..., (y + dy) mod H, (x + dx) mod W]."""
    return np.roll(a, shift=(-dy, -dx), axis=(-2, -1))


def conv3x3(x, w, b):
    """out[n, o, y, x] = b[o] + sum_{c, ky, kx} w[o, c, ky, kx] x[n, c, y + ky - 1, x + kx - 1]."""
    out = np.zeros((x.shape[0], w.shape[0]) + x.shape[2:])
    for ky in range(3):
        for kx in range(3):
            out += np.einsum("oc,nchw->nohw", w[:, :, ky, kx], _shift(x, ky - 1, kx - 1))
    return out + b[None, :, None, None]


def conv3x3_backward(x, w, gout):
    """Gradients of sum(gout * conv3x3(x, w, b)) with respect to x, w and b."""
    gx = np.zeros_like(x)
    gw = np.zeros_like(w)
    for ky in range(3):
        for kx in range(3):
            gw[:, :, ky, kx] = np.einsum("nohw,nchw->oc", gout, _shift(x, ky - 1, kx - 1))
            gx += _shift(np.einsum("oc,nohw->nchw", w[:, :, ky, kx], gout), 1 - ky, 1 - kx)
    return gx, gw, gout.sum(axis=(0, 2, 3))


def gelu(u):
    return 0.5 * u * (1.0 + erf(u / math.sqrt(2.0)))


def gelu_grad(u):
    cdf = 0.5 * (1.0 + erf(u / math.sqrt(2.0)))
    pdf = np.exp(-0.5 * u * u) / math.sqrt(2.0 * math.pi)
    return cdf + u * pdf


def init_params(rng, c0=2, width=64, layers=6):
    """He-style normal init scaled by 1/sqrt(9 Cin); the last layer is scaled by 0.1."""
    chans = [c0] + [width] * (layers - 1) + [c0]
    params = []
    for i in range(layers):
        cin, cout = chans[i], chans[i + 1]
        w = rng.standard_normal((cout, cin, 3, 3)) * math.sqrt(2.0 / (9 * cin))
        if i == layers - 1:
            w *= 0.1
        params.append((w, np.zeros(cout)))
    return params


def forward(params, x, keep=False):
    """y = x + net(x); with keep=True also returns the pre-activations and layer inputs."""
    h = x
    pre, ins = [], []
    for i, (w, b) in enumerate(params):
        ins.append(h)
        u = conv3x3(h, w, b)
        pre.append(u)
        h = gelu(u) if i < len(params) - 1 else u
    y = x + h
    return (y, pre, ins) if keep else y


def mse(y, target):
    return float(np.mean((y - target) ** 2))


def loss_and_grads(params, x, target):
    y, pre, ins = forward(params, x, keep=True)
    g = 2.0 * (y - target) / y.size          # d mse / d y (the residual path adds x, not params)
    grads = [None] * len(params)
    for i in reversed(range(len(params))):
        if i < len(params) - 1:
            g = g * gelu_grad(pre[i])
        gx, gw, gb = conv3x3_backward(ins[i], params[i][0], g)
        grads[i] = (gw, gb)
        g = gx
    return mse(y, target), grads


def adam_step(params, grads, state, lr, step, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (bias-corrected); `state` is a list of (m, v) pairs, updated in place."""
    out = []
    for i, ((w, b), (gw, gb)) in enumerate(zip(params, grads)):
        new = []
        for j, (p, g) in enumerate(((w, gw), (b, gb))):
            m, v = state[i][j]
            m[...] = beta1 * m + (1 - beta1) * g
            v[...] = beta2 * v + (1 - beta2) * g * g
            mh = m / (1 - beta1 ** step)
            vh = v / (1 - beta2 ** step)
            new.append(p - lr * mh / (np.sqrt(vh) + eps))
        out.append(tuple(new))
    return out


def flatten(params):
    """Parameters in the order layer by layer, weight (Cout, Cin, 3, 3) then bias."""
    return np.concatenate([np.concatenate([w.reshape(-1), b.reshape(-1)]) for w, b in params])


def unflatten(flat, c0=2, width=64, layers=6):
    chans = [c0] + [width] * (layers - 1) + [c0]
    out, k = [], 0
    for i in range(layers):
        cin, cout = chans[i], chans[i + 1]
        w = np.asarray(flat[k:k + cout * cin * 9], dtype=np.float64).reshape(cout, cin, 3, 3)
        k += cout * cin * 9
        b = np.asarray(flat[k:k + cout], dtype=np.float64)
        k += cout
        out.append((w, b))
    return out


def n_params(params):
    return sum(w.size + b.size for w, b in params)


def forward_flops(h, w, c0=2, width=64, layers=6):
    chans = [c0] + [width] * (layers - 1) + [c0]
    return sum(2 * h * w * 9 * chans[i] * chans[i + 1] for i in range(layers))
