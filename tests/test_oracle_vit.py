"""Pins of the FP64 ViT surrogate oracle (oracle/vit.py), independent of the GPU path:
central finite differences of the loss for every parameter tensor and the input, LayerNorm
moments, attention special cases (equal keys average the values; rows of the weights sum to
one), permutation equivariance of the blocks without positional embedding, blocks with zero
output projections reducing the model to embedding + head, the parameter count of the
Table II configuration, GELU's derivative and Adam's first step."""
import math

import numpy as np
import pytest

from oracle import vit as V

TINY = V.Config(channels=2, height=8, width=8, patch=2, layers=2, heads=2, embed=16,
                mlp_hidden=32)


def _tiny_params(rng, scale=0.3):
    flat = V.init_params(TINY, rng)
    flat += scale * rng.standard_normal(flat.size)   # away from the symmetric init
    return flat


def test_every_gradient_matches_central_differences():
    rng = np.random.default_rng(5)
    flat = _tiny_params(rng)
    x = rng.standard_normal((2, 2, 8, 8))
    target = rng.standard_normal((2, 2, 8, 8))
    L, g = V.loss_and_grad(TINY, flat, x, target)
    o = 0
    h = 1e-6
    for name, shape in V.param_shapes(TINY):
        n = int(np.prod(shape))
        for j in rng.choice(n, size=min(n, 4), replace=False):
            i = o + int(j)
            fp, fm = flat.copy(), flat.copy()
            fp[i] += h
            fm[i] -= h
            num = (V.loss(V.forward(TINY, fp, x)[0], target) -
                   V.loss(V.forward(TINY, fm, x)[0], target)) / (2 * h)
            assert abs(num - g[i]) <= 1e-6 * max(1e-3, abs(num)), (name, j, num, g[i])
        o += n
    # input gradient
    y, cache = V.forward(TINY, flat, x)
    dy = 2.0 * (y - target) / y.size
    _, dx = V.backward(TINY, flat, cache, dy)
    for idx in [(0, 0, 0, 0), (1, 1, 7, 3), (0, 1, 4, 5)]:
        xp, xm = x.copy(), x.copy()
        xp[idx] += h
        xm[idx] -= h
        num = (V.loss(V.forward(TINY, flat, xp)[0], target) -
               V.loss(V.forward(TINY, flat, xm)[0], target)) / (2 * h)
        assert abs(num - dx[idx]) <= 1e-6 * max(1e-3, abs(num))


def test_layernorm_rows_have_zero_mean_unit_variance():
    rng = np.random.default_rng(1)
    v = 3.0 + 2.0 * rng.standard_normal((5, 64))
    y, _ = V.layernorm(v, np.ones(64), np.zeros(64))
    assert np.allclose(y.mean(-1), 0.0, atol=1e-12)
    var = v.var(-1)
    assert np.allclose((y ** 2).mean(-1), var / (var + V.LN_EPS), rtol=1e-12)


def test_attention_with_equal_keys_averages_the_values():
    rng = np.random.default_rng(2)
    cfg = V.Config(embed=16, heads=2)
    B, T, D = 2, 6, 16
    qkv = rng.standard_normal((B, T, 3 * D))
    qkv[:, :, D:2 * D] = qkv[:, :1, D:2 * D]          # every token has the same key
    o, P = V.attention(cfg, qkv)
    assert np.allclose(P, 1.0 / T)
    assert np.allclose(o, qkv[:, :, 2 * D:].mean(axis=1, keepdims=True))
    # one key much closer to every query selects its value
    qkv = rng.standard_normal((B, T, 3 * D))
    qkv[:, 3, D:2 * D] = 1e3 * qkv[:, 0, :D]
    qkv[:, :, :D] = qkv[:, :1, :D]
    o, P = V.attention(cfg, qkv)
    assert np.allclose(P.sum(-1), 1.0)
    sel = qkv[:, 3, 2 * D:]
    assert np.allclose(o, sel[:, None, :], atol=1e-9)


def test_attention_scale_and_heads_closed_form():
    # two tokens, two heads of dh = 4: head 0 sees logits (a, 0) / sqrt(dh) -> weights
    # (sigmoid(a / 2), 1 - sigmoid(a / 2)); head 1 has equal keys -> the mean of its values
    cfg = V.Config(embed=8, heads=2)
    a = 1.7
    qkv = np.zeros((1, 2, 24))
    qkv[0, :, 0] = 1.0                     # q of head 0 = e0 for both tokens
    qkv[0, 0, 8] = a                       # k of token 0, head 0 = a e0; token 1 = 0
    qkv[0, :, 12:16] = [[0.3, 0, 0, 0], [0.3, 0, 0, 0]]   # equal keys in head 1
    qkv[0, :, 4] = 2.0                     # q of head 1
    vals = np.arange(16, dtype=float).reshape(2, 8)
    qkv[0, :, 16:24] = vals
    o, P = V.attention(cfg, qkv)
    w0 = 1.0 / (1.0 + math.exp(-a / 2.0))
    assert np.allclose(P[0, 0], [[w0, 1 - w0], [w0, 1 - w0]])
    assert np.allclose(P[0, 1], 0.5)
    assert np.allclose(o[0, :, :4], w0 * vals[0, :4] + (1 - w0) * vals[1, :4])
    assert np.allclose(o[0, :, 4:], vals[:, 4:].mean(axis=0))


def test_blocks_are_permutation_equivariant_without_positions():
    rng = np.random.default_rng(3)
    flat = _tiny_params(rng)
    V.unflatten(TINY, flat)["pos"][...] = 0.0
    x = rng.standard_normal((1, 2, 8, 8))
    perm = rng.permutation(TINY.tokens)
    xp = V.unpatchify(TINY, V.patchify(TINY, x)[:, perm])
    y, _ = V.forward(TINY, flat, x)
    yp, _ = V.forward(TINY, flat, xp)
    assert np.allclose(V.patchify(TINY, yp), V.patchify(TINY, y)[:, perm], atol=1e-12)


def test_zero_output_projections_leave_embedding_and_head():
    rng = np.random.default_rng(4)
    flat = _tiny_params(rng)
    p = V.unflatten(TINY, flat)
    for l in range(TINY.layers):
        for n in (f"W_o{l}", f"b_o{l}", f"W_2{l}", f"b_2{l}"):
            p[n][...] = 0.0
    x = rng.standard_normal((2, 2, 8, 8))
    y, _ = V.forward(TINY, flat, x)
    # the same map written out directly: patches -> embedding -> LayerNorm -> head
    pt = V.patchify(TINY, x)
    e = pt @ p["W_pe"].T + p["b_pe"] + p["pos"]
    z = (e - e.mean(-1, keepdims=True)) / np.sqrt(e.var(-1, keepdims=True) + V.LN_EPS)
    out = (z * p["lnf_g"] + p["lnf_b"]) @ p["W_h"].T + p["b_h"]
    assert np.allclose(y, x + V.unpatchify(TINY, out), atol=1e-12)


def test_patchify_roundtrip_and_order():
    x = np.arange(2 * 8 * 8, dtype=float).reshape(1, 2, 8, 8)
    pt = V.patchify(TINY, x)
    assert pt.shape == (1, 16, 8)
    # token 1 is the second 2x2 block of the first block row; channel 0 then channel 1
    assert list(pt[0, 1]) == [2, 3, 10, 11, 66, 67, 74, 75]
    assert np.array_equal(V.unpatchify(TINY, pt), x)


def test_table2_parameter_count():
    # D = 1024, F = 4096, P = 32, T = 256: embedding D P + D + T D, per layer
    # 12 D^2 + 13 D (two LayerNorms, qkv, projection, MLP), final LayerNorm and head
    D, F, P, T = 1024, 4096, 32, 256
    want = D * P + D + T * D + 12 * (4 * D + 3 * D * D + 3 * D + D * D + D + 2 * F * D + F + D) \
        + 2 * D + P * D + P
    assert V.num_params(V.TABLE2_64) == want == 151485472
    # the paper lists 157M for this row; the backbone it describes accounts for 96.5 %
    assert abs(want / 157e6 - 1.0) < 0.04


def test_gelu_derivative_and_adam_first_step():
    u = np.linspace(-4, 4, 41)
    h = 1e-6
    assert np.allclose(V.gelu_grad(u), (V.gelu(u + h) - V.gelu(u - h)) / (2 * h), atol=1e-8)
    assert abs(V.gelu(np.array([1.0]))[0] - 0.5 * (1 + math.erf(1 / math.sqrt(2)))) < 1e-15
    rng = np.random.default_rng(6)
    w = rng.standard_normal(10)
    g = rng.standard_normal(10)
    w1, m, v = V.adam(w, g, np.zeros(10), np.zeros(10), 1, lr=1e-2, eps=0.0)
    assert np.allclose(w1, w - 1e-2 * np.sign(g))
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)
