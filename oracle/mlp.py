"""FP64 CPU reference of the order-prediction network and its training step.

TEST INFRASTRUCTURE ONLY (used by the test-suite to check the GPU network
kernels).  Shares no code with the product library.

Network: 85 -> 128 -> 128 -> 57, ReLU after the two hidden layers; the 57
outputs are three groups (one per axis) of 19 class logits.  Loss per sample:
the sum over the three axes of the softmax cross-entropy; the batch loss is
the mean over samples.  Parameter vector layout: W1 [85][128], b1 [128],
W2 [128][128], b2 [128], W3 [128][57], b3 [57] (weights input-major:
y = x @ W + b).
"""
from __future__ import annotations

import numpy as np

IN, H, NCLS = 85, 128, 19
OUT = 3 * NCLS
SHAPES = [("W1", (IN, H)), ("b1", (H,)), ("W2", (H, H)), ("b2", (H,)), ("W3", (H, OUT)), ("b3", (OUT,))]
NPARAMS = sum(int(np.prod(s)) for _, s in SHAPES)


def unpack(p):
    p = np.asarray(p, dtype=np.float64)
    out, o = {}, 0
    for name, shape in SHAPES:
        n = int(np.prod(shape))
        out[name] = p[o:o + n].reshape(shape)
        o += n
    return out


def pack(d):
    return np.concatenate([np.asarray(d[name], dtype=np.float64).reshape(-1) for name, _ in SHAPES])


def forward(p, x):
    """Logits [B][57] and the hidden activations."""
    w = unpack(p)
    x = np.asarray(x, dtype=np.float64)
    h1 = np.maximum(x @ w["W1"] + w["b1"], 0.0)
    h2 = np.maximum(h1 @ w["W2"] + w["b2"], 0.0)
    z = h2 @ w["W3"] + w["b3"]
    return z, h1, h2


def loss_and_grad(p, x, labels):
    """(sum over the batch of per-sample losses, gradient of the MEAN loss)."""
    w = unpack(p)
    x = np.asarray(x, dtype=np.float64)
    labels = np.asarray(labels)
    B = x.shape[0]
    z, h1, h2 = forward(p, x)
    loss = 0.0
    dz = np.zeros_like(z)
    for ax in range(3):
        zz = z[:, ax * NCLS:(ax + 1) * NCLS]
        zz = zz - zz.max(axis=1, keepdims=True)
        e = np.exp(zz)
        pr = e / e.sum(axis=1, keepdims=True)
        y = labels[:, ax]
        loss += float(-np.log(pr[np.arange(B), y]).sum())
        oh = np.zeros_like(pr)
        oh[np.arange(B), y] = 1.0
        dz[:, ax * NCLS:(ax + 1) * NCLS] = (pr - oh) / B
    g = {}
    g["W3"] = h2.T @ dz
    g["b3"] = dz.sum(0)
    dh2 = (dz @ w["W3"].T) * (h2 > 0)
    g["W2"] = h1.T @ dh2
    g["b2"] = dh2.sum(0)
    dh1 = (dh2 @ w["W2"].T) * (h1 > 0)
    g["W1"] = x.T @ dh1
    g["b1"] = dh1.sum(0)
    return loss, pack(g)


def adam(p, g, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (Kingma & Ba): returns new (p, m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


def choose(z, p_cover, kmin=6):
    """Per axis, the smallest K whose cumulative softmax probability
    reaches p_cover."""
    z = np.asarray(z, dtype=np.float64)
    out = np.zeros((z.shape[0], 3), dtype=np.int32)
    for ax in range(3):
        zz = z[:, ax * NCLS:(ax + 1) * NCLS]
        e = np.exp(zz - zz.max(axis=1, keepdims=True))
        cdf = np.cumsum(e / e.sum(axis=1, keepdims=True), axis=1)
        idx = np.argmax(cdf >= p_cover, axis=1)
        idx[~(cdf >= p_cover).any(axis=1)] = NCLS - 1
        out[:, ax] = kmin + idx
    return out
