"""FP64 oracle of the vision-transformer forecast surrogate (test infrastructure only).

Architecture (Sec. III-B, Fig. `fig:arch`, Table II): a standard ViT backbone over the
state image.  A C x H x W state is cut into non-overlapping p x p patches, T = (H/p)(W/p)
tokens, each patch flattened in (channel, row, column) order to P = C p^2 values.
  tokens   h0 = patches W_pe^T + b_pe + pos                       (linear patch embedding,
                                                                    learned positions)
  block l  a  = LN1(h);  [q|k|v] = a W_qkv^T + b_qkv              (pre-norm, D = heads x dh)
           o  = concat_heads softmax(q k^T / sqrt(dh)) v;  h = h + o W_o^T + b_o
           m  = LN2(h);  h = h + gelu(m W_1^T + b_1) W_2^T + b_2   (exact erf-GELU, MLP
                                                                    hidden = ratio x D)
  head     out = LNf(h) W_h^T + b_h  (T x P), unpatchified; prediction y = x + out.
LayerNorm: (v - mean) / sqrt(var + 1e-5) * gamma + beta over the features of a token,
population variance.  Dropout and DropPath (the paper's regularisers) are off: they do not
change the compute path and keep forward and gradients deterministic.
Loss: mean squared error over all outputs; optimiser: Adam (Kingma & Ba, 2015) on FP32
master weights.

Parameters travel flat in this order (the library's ABI order): W_pe (D, P), b_pe (D),
pos (T, D); per layer: ln1 gamma, beta (D), W_qkv (3D, D), b_qkv (3D), W_o (D, D), b_o (D),
ln2 gamma, beta (D), W_1 (F, D), b_1 (F), W_2 (D, F), b_2 (D); then lnf gamma, beta (D),
W_h (P, D), b_h (P).  Weights are (out, in): y = v W^T + b.

The backward pass is written out by hand, operation by operation in reverse; it is pinned by
central finite differences of the loss (tests/test_oracle_vit.py).
"""
import math
from dataclasses import dataclass

import numpy as np
from scipy.special import erf

LN_EPS = 1e-5


@dataclass(frozen=True)
class Config:
    channels: int = 2
    height: int = 64
    width: int = 64
    patch: int = 4
    layers: int = 12
    heads: int = 8
    embed: int = 1024
    mlp_hidden: int = 4096

    @property
    def tokens(self):
        return (self.height // self.patch) * (self.width // self.patch)

    @property
    def patch_dim(self):
        return self.channels * self.patch * self.patch

    @property
    def head_dim(self):
        return self.embed // self.heads


# Table II, first row: 64^2 input, patch 4, 12 layers, 8 heads, embed 1024, MLP ratio 4
TABLE2_64 = Config()


def param_shapes(cfg):
    """(name, shape) of every parameter tensor in ABI order."""
    D, F, P, T = cfg.embed, cfg.mlp_hidden, cfg.patch_dim, cfg.tokens
    out = [("W_pe", (D, P)), ("b_pe", (D,)), ("pos", (T, D))]
    for l in range(cfg.layers):
        out += [(f"ln1_g{l}", (D,)), (f"ln1_b{l}", (D,)),
                (f"W_qkv{l}", (3 * D, D)), (f"b_qkv{l}", (3 * D,)),
                (f"W_o{l}", (D, D)), (f"b_o{l}", (D,)),
                (f"ln2_g{l}", (D,)), (f"ln2_b{l}", (D,)),
                (f"W_1{l}", (F, D)), (f"b_1{l}", (F,)),
                (f"W_2{l}", (D, F)), (f"b_2{l}", (D,))]
    out += [("lnf_g", (D,)), ("lnf_b", (D,)), ("W_h", (P, D)), ("b_h", (P,))]
    return out


def num_params(cfg):
    return int(sum(np.prod(s) for _, s in param_shapes(cfg)))


def unflatten(cfg, flat):
    """Dict of views into the flat parameter vector."""
    out, o = {}, 0
    for name, shape in param_shapes(cfg):
        n = int(np.prod(shape))
        out[name] = flat[o:o + n].reshape(shape)
        o += n
    assert o == flat.size
    return out


def init_params(cfg, rng):
    """Normal(0, 0.02) weights and positions, zero biases, unit LayerNorm gains; the
    output head scaled by 0.1 so the untrained model starts near the identity map."""
    flat = np.zeros(num_params(cfg))
    p = unflatten(cfg, flat)
    for name, shape in param_shapes(cfg):
        if name.startswith(("W_", "pos")):
            p[name][...] = 0.02 * rng.standard_normal(shape)
        elif name.startswith(("ln1_g", "ln2_g", "lnf_g")):
            p[name][...] = 1.0
    p["W_h"][...] *= 0.1
    return flat


# ------------------------------------------------------------------------------------------
# pieces

def patchify(cfg, x):
    """x (B, C, H, W) -> (B, T, P); token t = (row block, column block) in row-major
    order, patch values in (channel, row in patch, column in patch) order."""
    B, C, H, W = x.shape
    p = cfg.patch
    v = x.reshape(B, C, H // p, p, W // p, p)          # b c ty py tx px
    v = v.transpose(0, 2, 4, 1, 3, 5)                  # b ty tx c py px
    return v.reshape(B, (H // p) * (W // p), C * p * p)


def unpatchify(cfg, tok):
    """Inverse of patchify: (B, T, P) -> (B, C, H, W)."""
    B = tok.shape[0]
    C, H, W, p = cfg.channels, cfg.height, cfg.width, cfg.patch
    v = tok.reshape(B, H // p, W // p, C, p, p)        # b ty tx c py px
    v = v.transpose(0, 3, 1, 4, 2, 5)                  # b c ty py tx px
    return v.reshape(B, C, H, W)


def layernorm(v, g, b):
    mu = v.mean(axis=-1, keepdims=True)
    var = ((v - mu) ** 2).mean(axis=-1, keepdims=True)
    rstd = 1.0 / np.sqrt(var + LN_EPS)
    xhat = (v - mu) * rstd
    return xhat * g + b, (xhat, rstd)


def layernorm_backward(dy, cache, g):
    """Gradients of sum(dy * LN(v)) with respect to v, gamma and beta."""
    xhat, rstd = cache
    dxhat = dy * g
    n = xhat.shape[-1]
    dv = rstd * (dxhat - dxhat.sum(-1, keepdims=True) / n
                 - xhat * (dxhat * xhat).sum(-1, keepdims=True) / n)
    red = tuple(range(dy.ndim - 1))
    return dv, (dy * xhat).sum(axis=red), dy.sum(axis=red)


def gelu(u):
    return 0.5 * u * (1.0 + erf(u / math.sqrt(2.0)))


def gelu_grad(u):
    cdf = 0.5 * (1.0 + erf(u / math.sqrt(2.0)))
    pdf = np.exp(-0.5 * u * u) / math.sqrt(2.0 * math.pi)
    return cdf + u * pdf


def softmax(s):
    e = np.exp(s - s.max(axis=-1, keepdims=True))
    return e / e.sum(axis=-1, keepdims=True)


def attention(cfg, qkv):
    """qkv (B, T, 3D) -> o (B, T, D) and the weights (B, heads, T, T)."""
    B, T, _ = qkv.shape
    D, H, dh = cfg.embed, cfg.heads, cfg.head_dim
    q = qkv[..., :D].reshape(B, T, H, dh).transpose(0, 2, 1, 3)
    k = qkv[..., D:2 * D].reshape(B, T, H, dh).transpose(0, 2, 1, 3)
    v = qkv[..., 2 * D:].reshape(B, T, H, dh).transpose(0, 2, 1, 3)
    P = softmax(q @ k.transpose(0, 1, 3, 2) / math.sqrt(dh))
    o = (P @ v).transpose(0, 2, 1, 3).reshape(B, T, D)
    return o, P


def attention_backward(cfg, qkv, P, do):
    """Gradient of sum(do * attention(qkv)) with respect to qkv."""
    B, T, _ = qkv.shape
    D, H, dh = cfg.embed, cfg.heads, cfg.head_dim
    split = lambda a: a.reshape(B, T, H, dh).transpose(0, 2, 1, 3)
    q, k, v = split(qkv[..., :D]), split(qkv[..., D:2 * D]), split(qkv[..., 2 * D:])
    dO = split(do)
    dv = P.transpose(0, 1, 3, 2) @ dO
    dP = dO @ v.transpose(0, 1, 3, 2)
    dS = P * (dP - (dP * P).sum(axis=-1, keepdims=True)) / math.sqrt(dh)
    dq = dS @ k
    dk = dS.transpose(0, 1, 3, 2) @ q
    merge = lambda a: a.transpose(0, 2, 1, 3).reshape(B, T, D)
    return np.concatenate([merge(dq), merge(dk), merge(dv)], axis=-1)


def linear(v, W, b):
    return v @ W.T + b


# ------------------------------------------------------------------------------------------
# model

def forward(cfg, flat, x):
    """Prediction y = x + out(x) for x (B, C, H, W) and the cache the backward pass needs."""
    p = unflatten(cfg, flat)
    pt = patchify(cfg, x)
    h = linear(pt, p["W_pe"], p["b_pe"]) + p["pos"]
    cache = {"pt": pt, "layers": []}
    for l in range(cfg.layers):
        c = {"h_in": h}
        a, c["ln1"] = layernorm(h, p[f"ln1_g{l}"], p[f"ln1_b{l}"])
        qkv = linear(a, p[f"W_qkv{l}"], p[f"b_qkv{l}"])
        o, P = attention(cfg, qkv)
        h = h + linear(o, p[f"W_o{l}"], p[f"b_o{l}"])
        m, c["ln2"] = layernorm(h, p[f"ln2_g{l}"], p[f"ln2_b{l}"])
        u = linear(m, p[f"W_1{l}"], p[f"b_1{l}"])
        g = gelu(u)
        h = h + linear(g, p[f"W_2{l}"], p[f"b_2{l}"])
        c.update(a=a, qkv=qkv, P=P, o=o, m=m, u=u, g=g)
        cache["layers"].append(c)
    f, cache["lnf"] = layernorm(h, p["lnf_g"], p["lnf_b"])
    cache["f"] = f
    out = linear(f, p["W_h"], p["b_h"])
    return x + unpatchify(cfg, out), cache


def loss(y, target):
    return float(np.mean((y - target) ** 2))


def backward(cfg, flat, cache, dy):
    """Gradients of sum(dy * forward(x)) with respect to the flat parameters and to x."""
    p = unflatten(cfg, flat)
    grad = np.zeros_like(flat)
    gp = unflatten(cfg, grad)
    dout = patchify(cfg, dy)                               # head output, (B, T, P)
    gp["W_h"][...] = np.einsum("btp,btd->pd", dout, cache["f"])
    gp["b_h"][...] = dout.sum(axis=(0, 1))
    df = dout @ p["W_h"]
    dh, gp["lnf_g"][...], gp["lnf_b"][...] = layernorm_backward(df, cache["lnf"], p["lnf_g"])
    for l in reversed(range(cfg.layers)):
        c = cache["layers"][l]
        # MLP sub-block: h_out = h_mid + gelu(m W_1^T + b_1) W_2^T + b_2
        gp[f"W_2{l}"][...] = np.einsum("btd,btf->df", dh, c["g"])
        gp[f"b_2{l}"][...] = dh.sum(axis=(0, 1))
        du = (dh @ p[f"W_2{l}"]) * gelu_grad(c["u"])
        gp[f"W_1{l}"][...] = np.einsum("btf,btd->fd", du, c["m"])
        gp[f"b_1{l}"][...] = du.sum(axis=(0, 1))
        dm = du @ p[f"W_1{l}"]
        dln, gp[f"ln2_g{l}"][...], gp[f"ln2_b{l}"][...] = layernorm_backward(
            dm, c["ln2"], p[f"ln2_g{l}"])
        dh = dh + dln
        # attention sub-block: h_mid = h_in + attn(LN1(h_in)) W_o^T + b_o
        gp[f"W_o{l}"][...] = np.einsum("btd,bte->de", dh, c["o"])
        gp[f"b_o{l}"][...] = dh.sum(axis=(0, 1))
        do = dh @ p[f"W_o{l}"]
        dqkv = attention_backward(cfg, c["qkv"], c["P"], do)
        gp[f"W_qkv{l}"][...] = np.einsum("btj,btd->jd", dqkv, c["a"])
        gp[f"b_qkv{l}"][...] = dqkv.sum(axis=(0, 1))
        da = dqkv @ p[f"W_qkv{l}"]
        dln, gp[f"ln1_g{l}"][...], gp[f"ln1_b{l}"][...] = layernorm_backward(
            da, c["ln1"], p[f"ln1_g{l}"])
        dh = dh + dln
    gp["pos"][...] = dh.sum(axis=0)
    gp["W_pe"][...] = np.einsum("btd,btp->dp", dh, cache["pt"])
    gp["b_pe"][...] = dh.sum(axis=(0, 1))
    dx = dy + unpatchify(cfg, dh @ p["W_pe"])
    return grad, dx


def loss_and_grad(cfg, flat, x, target):
    y, cache = forward(cfg, flat, x)
    dy = 2.0 * (y - target) / y.size
    grad, _ = backward(cfg, flat, cache, dy)
    return loss(y, target), grad


def adam(flat, grad, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step (step counts from 1) on copies of (flat, m, v)."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mhat = m / (1.0 - beta1 ** step)
    vhat = v / (1.0 - beta2 ** step)
    return flat - lr * mhat / (np.sqrt(vhat) + eps), m, v


def training_flops(cfg, batch):
    """Matrix-product flops of one training step on `batch` states, 2 per multiply-add: the
    forward products, and in the backward pass the weight gradients of every linear layer
    and the input gradients of all but the patch embedding (whose input is data).  Apart
    from that embedding this is 3x the forward (eq. 18 counts 6 per token and parameter for
    the same reason).  Attention's two batched products per head are included (4 in the
    backward pass)."""
    T, D, F, P = cfg.tokens, cfg.embed, cfg.mlp_hidden, cfg.patch_dim
    body = cfg.layers * (3 * D * D + D * D + 2 * D * F) + D * P      # blocks and head
    per_token = 3 * 2 * body + 2 * 2 * P * D                         # + patch embedding
    attn = 3 * cfg.layers * 2 * 2 * T * T * D                        # q k^T and P v
    return batch * (T * per_token + attn)
