"""FP64 CPU oracle of the learned surrogate (not from the paper).

TEST INFRASTRUCTURE ONLY -- used by tests/ and never by the product path;
shares no code with the HIP kernels.

Network: six 3x3 convolutions with periodic (circular) padding, 32 channels,
ReLU after the first five.  Input: the RGB image f plus a constant lambda
map and a constant p map (5 channels).  Output: v = f + z6 (the network
predicts the correction to f; residual form).  Loss: mean squared error
against the plain ILS output.  Optimiser: Adam (Kingma & Ba, 2015) with
bias correction.

Convolution convention (cross-correlation, as in common deep-learning
libraries):  z[co, y, x] = b[co] + sum_{ci, a, c} w[co, ci, a, c] *
x[ci, (y + a - 1) mod H, (x + c - 1) mod W].

Parity status: pinned -- the convolution against scipy.ndimage.correlate
(mode="wrap"), the gradients against central finite differences of the
loss, Adam against its closed-form first step.
"""
from __future__ import annotations

import numpy as np

CH = 32
LAYERS = [(5, CH), (CH, CH), (CH, CH), (CH, CH), (CH, CH), (CH, 3)]


def init_params(seed: int = 0):
    """He-style initialisation; the last layer starts small so v ~ f."""
    rng = np.random.default_rng(seed)
    params = []
    for i, (ci, co) in enumerate(LAYERS):
        std = np.sqrt(2.0 / (9 * ci))
        if i == len(LAYERS) - 1:
            std *= 0.1
        params.append({"w": rng.standard_normal((co, ci, 3, 3)) * std, "b": np.zeros(co)})
    return params


def net_input(f, lam, p):
    """(3, H, W) image + constant lambda and p maps -> (5, H, W)."""
    f = np.asarray(f, dtype=np.float64)
    H, W = f.shape[-2:]
    return np.concatenate([f, np.full((1, H, W), lam), np.full((1, H, W), p)], axis=0)


def conv3x3(x, w, b):
    """Periodic 3x3 cross-correlation: x (Ci, H, W), w (Co, Ci, 3, 3)."""
    out = np.zeros((w.shape[0],) + x.shape[1:])
    for a in range(3):
        for c in range(3):
            xs = np.roll(np.roll(x, -(a - 1), axis=1), -(c - 1), axis=2)  # xs[y, x] = x[y+a-1, x+c-1]
            out += np.einsum("oi,ihw->ohw", w[:, :, a, c], xs)
    return out + b[:, None, None]


def conv3x3_grad_input(g, w):
    """d(loss)/dx given g = d(loss)/dz for z = conv3x3(x, w, b)."""
    dx = np.zeros((w.shape[1],) + g.shape[1:])
    for a in range(3):
        for c in range(3):
            t = np.einsum("oi,ohw->ihw", w[:, :, a, c], g)
            dx += np.roll(np.roll(t, a - 1, axis=1), c - 1, axis=2)  # x[y'] receives g[y' - a + 1]
    return dx


def conv3x3_grad_weight(g, x):
    """d(loss)/dw and d(loss)/db for z = conv3x3(x, w, b)."""
    dw = np.zeros((g.shape[0], x.shape[0], 3, 3))
    for a in range(3):
        for c in range(3):
            xs = np.roll(np.roll(x, -(a - 1), axis=1), -(c - 1), axis=2)
            dw[:, :, a, c] = np.einsum("ohw,ihw->oi", g, xs)
    return dw, g.sum(axis=(1, 2))


def forward(params, x, f):
    """Returns v and the activations needed by backward."""
    acts = [x]
    a = x
    for i, prm in enumerate(params):
        z = conv3x3(a, prm["w"], prm["b"])
        if i < len(params) - 1:
            a = np.maximum(z, 0.0)
        else:
            a = z
        acts.append(a)
    return np.asarray(f, dtype=np.float64) + acts[-1], acts


def mse(v, t):
    return float(np.mean((v - t) ** 2))


def backward(params, acts, v, t):
    """Gradients of mse(v, t) w.r.t. every w and b (list of dicts)."""
    g = 2.0 * (v - t) / v.size  # d loss / d z6  (v = f + z6)
    grads = [None] * len(params)
    for i in range(len(params) - 1, -1, -1):
        dw, db = conv3x3_grad_weight(g, acts[i])
        grads[i] = {"w": dw, "b": db}
        if i > 0:
            g = conv3x3_grad_input(g, params[i]["w"]) * (acts[i] > 0)
    return grads


def adam_init(params):
    return {"t": 0, "m": [{k: np.zeros_like(v) for k, v in p.items()} for p in params],
            "v": [{k: np.zeros_like(v) for k, v in p.items()} for p in params]}


def adam_step(params, grads, state, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """theta -= lr * mhat / (sqrt(vhat) + eps), with m, v the biased moments."""
    state["t"] += 1
    t = state["t"]
    for p, g, m, v in zip(params, grads, state["m"], state["v"]):
        for k in p:
            m[k] = b1 * m[k] + (1 - b1) * g[k]
            v[k] = b2 * v[k] + (1 - b2) * g[k] ** 2
            mhat = m[k] / (1 - b1 ** t)
            vhat = v[k] / (1 - b2 ** t)
            p[k] = p[k] - lr * mhat / (np.sqrt(vhat) + eps)
    return params


def bf16_round(a):
    """Round float values to bfloat16 (nearest, ties to even), returned as float64."""
    a32 = np.asarray(a, dtype=np.float32)
    u = a32.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)
