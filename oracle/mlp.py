"""CPU oracle of the learned scheduler's network (test infrastructure only).

Only tests/, __graft_entry__.smoke() and bench.py's cpu_baseline leg use this
module; the product path never imports it.

The network is not part of the paper (which names an adaptive scheduler as
future work, Section 7): 12 round features -> 64 -> 64 -> 5 outputs with
ReLU hidden layers; weights, inputs and hidden activations are rounded to
bfloat16 (round to nearest even), products accumulate in higher precision.
Outputs: push logit, dense logit, three delta-class logits.  The loss is the
batch mean of two logistic losses (push, dense) and a softmax cross-entropy
(delta class).  Everything here is float64 apart from the bf16 rounding
points, written as plain loops over layers with numpy products.

Parameter block (float32[5317], row-major): W1[64][12], b1[64], W2[64][64],
b2[64], W3[5][64], b3[5].
"""
from __future__ import annotations

import numpy as np

NI, NH, NO = 12, 64, 5
SHAPES = [("W1", (NH, NI)), ("b1", (NH,)), ("W2", (NH, NH)), ("b2", (NH,)), ("W3", (NO, NH)), ("b3", (NO,))]
NPAR = sum(int(np.prod(s)) for _, s in SHAPES)


def unpack(p):
    out, k = {}, 0
    for name, shape in SHAPES:
        size = int(np.prod(shape))
        out[name] = np.asarray(p[k:k + size], dtype=np.float64).reshape(shape)
        k += size
    return out


def pack(d):
    return np.concatenate([np.asarray(d[name], np.float64).ravel() for name, _ in SHAPES])


def bf16(x):
    """Round float32 values to bfloat16 (nearest, ties to even), returned as float64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    finite = (u & 0x7F800000) != 0x7F800000
    lsb = (u >> 16) & 1
    r = np.where(finite, (u + 0x7FFF + lsb) & 0xFFFF0000, u & 0xFFFF0000)
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def _rnd(rounding):
    return bf16 if rounding else (lambda v: np.asarray(v, np.float64))


def layer1(p, x, rounding=True):
    """h1 = bf16(relu(W1 bf16(x) + b1))."""
    q, rnd = unpack(p), _rnd(rounding)
    return rnd(np.maximum(rnd(np.asarray(x, np.float64)) @ rnd(q["W1"]).T + rnd(q["b1"]), 0.0))


def layer2(p, h1, rounding=True):
    """h2 = bf16(relu(W2 h1 + b2))."""
    q, rnd = unpack(p), _rnd(rounding)
    return rnd(np.maximum(np.asarray(h1, np.float64) @ rnd(q["W2"]).T + rnd(q["b2"]), 0.0))


def layer3(p, h2, rounding=True):
    """logits = W3 h2 + b3."""
    q, rnd = unpack(p), _rnd(rounding)
    return np.asarray(h2, np.float64) @ rnd(q["W3"]).T + rnd(q["b3"])


def forward(p, x, rounding=True):
    """logits[B, 5], h1[B, 64], h2[B, 64] for inputs x[B, 12]."""
    h1 = layer1(p, x, rounding)
    h2 = layer2(p, h1, rounding)
    return layer3(p, h2, rounding), h1, h2


def targets(labels):
    """(push, dense, delta class) from round codes: mode in bits 0-1, class in bits 8-9."""
    labels = np.asarray(labels, np.int64)
    mode = labels & 3
    dc = np.minimum((labels >> 8) & 3, 2)
    return (mode == 2).astype(np.float64), (mode == 1).astype(np.float64), dc


def loss(logits, labels):
    """(mean loss, dloss/dlogits)."""
    z = np.asarray(logits, np.float64)
    B = z.shape[0]
    y0, y1, dc = targets(labels)
    total = 0.0
    d = np.zeros_like(z)
    for k, y in ((0, y0), (1, y1)):
        s = 1.0 / (1.0 + np.exp(-z[:, k]))
        total += np.sum(np.logaddexp(0.0, z[:, k]) - z[:, k] * y)
        d[:, k] = (s - y) / B
    zs = z[:, 2:5]
    mx = zs.max(axis=1, keepdims=True)
    e = np.exp(zs - mx)
    sm = e / e.sum(axis=1, keepdims=True)
    lse = mx[:, 0] + np.log(e.sum(axis=1))
    total += np.sum(lse - zs[np.arange(B), dc])
    onehot = np.zeros_like(zs)
    onehot[np.arange(B), dc] = 1.0
    d[:, 2:5] = (sm - onehot) / B
    return total / B, d


def backward(p, x, h1, h2, dlogits, rounding=True):
    """Gradient of sum(dlogits * logits) with respect to the parameters, given
    the forward pass's hidden activations h1, h2 (straight through the bf16
    rounding of weights and activations)."""
    q = unpack(p)
    rnd = bf16 if rounding else (lambda v: np.asarray(v, np.float64))
    W2, W3 = rnd(q["W2"]), rnd(q["W3"])
    x = rnd(np.asarray(x, np.float64))
    d = np.asarray(dlogits, np.float64)
    g = {"W3": d.T @ h2, "b3": d.sum(axis=0)}
    dz2 = (d @ W3) * (h2 > 0)
    g["W2"] = dz2.T @ h1
    g["b2"] = dz2.sum(axis=0)
    dz1 = (dz2 @ W2) * (h1 > 0)
    g["W1"] = dz1.T @ x
    g["b1"] = dz1.sum(axis=0)
    return pack(g)


def adam(g, p, m1, m2, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (bias-corrected); returns new (p, m1, m2)."""
    m1 = b1 * m1 + (1 - b1) * g
    m2 = b2 * m2 + (1 - b2) * g * g
    mh = m1 / (1 - b1 ** step)
    vh = m2 / (1 - b2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m1, m2

