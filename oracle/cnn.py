"""FP64 oracle of the tile-proposal CNN -- TEST INFRASTRUCTURE.

Nothing in the paper is learned; this network is an addition of this library, so the
oracle follows plain textbook definitions and is pinned by finite differences, by a
library convolution and by the zero-weight special case.

Network: L layers of 3x3 convolution (cross-correlation, zero padding 1, stride 1)
with bias; ReLU after every layer but the last; the last layer has one output
channel, the tile-logit map z[b][h][w]. Loss: softmax over all H*W tiles of a sample
and cross-entropy against a label distribution q (sums to 1), averaged over the batch:
    loss = -(1/B) sum_b sum_t q[b, t] log softmax(z[b])[t],   dloss/dz = (softmax - q) / B.
Parameters are one flat vector [W0, b0, W1, b1, ...], W_l laid out [C_out][C_in][3][3].
Adam: m = b1 m + (1-b1) g; v = b2 v + (1-b2) g^2; w -= lr (m / (1-b1^t)) / (sqrt(v / (1-b2^t)) + eps).
"""
from __future__ import annotations

from typing import List, Sequence, Tuple

import numpy as np


def layer_shapes(in_ch: int, hidden: int, layers: int) -> List[Tuple[int, int]]:
    """(C_in, C_out) of every layer."""
    chans = [in_ch] + [hidden] * (layers - 1) + [1]
    return [(chans[i], chans[i + 1]) for i in range(layers)]


def n_params(in_ch: int, hidden: int, layers: int) -> int:
    return sum(co * ci * 9 + co for ci, co in layer_shapes(in_ch, hidden, layers))


def unpack(theta: np.ndarray, in_ch: int, hidden: int, layers: int):
    out, o = [], 0
    for ci, co in layer_shapes(in_ch, hidden, layers):
        W = theta[o:o + co * ci * 9].reshape(co, ci, 3, 3)
        o += co * ci * 9
        b = theta[o:o + co]
        o += co
        out.append((W, b))
    assert o == theta.size
    return out


def conv3x3(x: np.ndarray, W: np.ndarray, b: np.ndarray) -> np.ndarray:
    """y[b, o, h, w] = b[o] + sum_{c, dy, dx} W[o, c, dy, dx] x[b, c, h + dy - 1, w + dx - 1]."""
    B, C, H, Wd = x.shape
    xp = np.zeros((B, C, H + 2, Wd + 2))
    xp[:, :, 1:-1, 1:-1] = x
    y = np.zeros((B, W.shape[0], H, Wd)) + b[None, :, None, None]
    for dy in range(3):
        for dx in range(3):
            patch = xp[:, :, dy:dy + H, dx:dx + Wd]                 # [B, C, H, W]
            y += np.einsum("oc,bchw->bohw", W[:, :, dy, dx], patch)
    return y


def forward(theta: np.ndarray, x: np.ndarray, in_ch: int, hidden: int, layers: int):
    """Returns (logits [B, H, W], cache of layer inputs and pre-activations)."""
    params = unpack(np.asarray(theta, dtype=np.float64), in_ch, hidden, layers)
    a = np.asarray(x, dtype=np.float64)
    cache = []
    for li, (W, b) in enumerate(params):
        z = conv3x3(a, W, b)
        cache.append((a, z))
        a = np.maximum(z, 0.0) if li < layers - 1 else z
    return a[:, 0], cache


def softmax_ce(z: np.ndarray, q: np.ndarray):
    """Mean cross-entropy over the batch and its gradient wrt the logits."""
    B = z.shape[0]
    zf = z.reshape(B, -1)
    qf = q.reshape(B, -1)
    m = zf.max(axis=1, keepdims=True)
    e = np.exp(zf - m)
    s = e.sum(axis=1, keepdims=True)
    logp = zf - m - np.log(s)
    loss = -np.sum(qf * logp) / B
    p = e / s
    return loss, ((p - qf) / B).reshape(z.shape), p.reshape(z.shape)


def backward(theta: np.ndarray, cache, dz: np.ndarray, in_ch: int, hidden: int, layers: int) -> np.ndarray:
    """Gradient of the loss wrt the flat parameter vector, given dloss/dlogits."""
    params = unpack(np.asarray(theta, dtype=np.float64), in_ch, hidden, layers)
    grads = []
    g = dz[:, None]                                                 # dloss/d(output of last layer)
    for li in range(layers - 1, -1, -1):
        W, b = params[li]
        a, z = cache[li]
        if li < layers - 1:
            g = g * (z > 0)                                         # through the ReLU
        B, C, H, Wd = a.shape
        ap = np.zeros((B, C, H + 2, Wd + 2))
        ap[:, :, 1:-1, 1:-1] = a
        dW = np.zeros_like(W)
        for dy in range(3):
            for dx in range(3):
                dW[:, :, dy, dx] = np.einsum("bohw,bchw->oc", g, ap[:, :, dy:dy + H, dx:dx + Wd])
        db = g.sum(axis=(0, 2, 3))
        grads.append((dW, db))
        # input gradient: full correlation with the flipped kernel
        gp = np.zeros((B, W.shape[0], H + 2, Wd + 2))
        gp[:, :, 1:-1, 1:-1] = g
        da = np.zeros_like(a)
        for dy in range(3):
            for dx in range(3):
                da += np.einsum("oc,bohw->bchw", W[:, :, 2 - dy, 2 - dx], gp[:, :, dy:dy + H, dx:dx + Wd])
        g = da
    out = []
    for dW, db in reversed(grads):
        out += [dW.ravel(), db]
    return np.concatenate(out)


def adam(theta, m, v, g, t: int, lr: float, b1: float = 0.9, b2: float = 0.999, eps: float = 1e-8):
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def he_init(in_ch: int, hidden: int, layers: int, seed: int) -> np.ndarray:
    """He-normal weights, zero biases (numpy PCG64 seeded)."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence(seed)))
    out = []
    for ci, co in layer_shapes(in_ch, hidden, layers):
        out += [rng.standard_normal(co * ci * 9) * np.sqrt(2.0 / (ci * 9)), np.zeros(co)]
    return np.concatenate(out)
