"""Float64 reference of the node-proposal network: forward, hand-written
backward, Adam.

TEST INFRASTRUCTURE ONLY (see the package header).  Not from the paper (the
learned shortened quadrature is an addition on top of the method); pinned in
the tests by central finite differences of the loss.

Parameters are one flat vector [W1, b1, W2, b2, W3, b3, W4, b4] with
W_l of shape (out, in) row-major; sizes 6 -> 64 -> 64 -> 64 -> 65; the three
hidden layers use GELU(x) = x Phi(x) = x (1 + erf(x / sqrt 2)) / 2, the output
layer is linear.
"""
from __future__ import annotations

import numpy as np
from scipy import special

SIZES = (6, 64, 64, 64, 65)


def unpack(params, sizes=SIZES):
    p = np.asarray(params, dtype=np.float64)
    out, o = [], 0
    for i, j in zip(sizes[:-1], sizes[1:]):
        W = p[o:o + i * j].reshape(j, i)
        o += i * j
        b = p[o:o + j]
        o += j
        out.append((W, b))
    assert o == p.size
    return out


def gelu(x):
    return 0.5 * x * (1.0 + special.erf(x / np.sqrt(2.0)))


def gelu_grad(x):
    return 0.5 * (1.0 + special.erf(x / np.sqrt(2.0))) + x * np.exp(-0.5 * x * x) / np.sqrt(2.0 * np.pi)


def forward(params, X):
    """X: (B, 6).  Returns (Y (B, 65), cache of pre-activations)."""
    layers = unpack(params)
    a = np.asarray(X, dtype=np.float64)
    pre = []
    for li, (W, b) in enumerate(layers):
        z = a @ W.T + b
        if li < len(layers) - 1:
            pre.append(z)
            a = gelu(z)
        else:
            a = z
    return a, (np.asarray(X, dtype=np.float64), pre)


def backward(params, cache, dY):
    """Gradient of sum_b <dY_b, Y_b> with respect to the flat parameters."""
    layers = unpack(params)
    X, pre = cache
    acts = [X] + [gelu(z) for z in pre]
    grads = [None] * len(layers)
    d = np.asarray(dY, dtype=np.float64)
    for li in range(len(layers) - 1, -1, -1):
        W, _b = layers[li]
        grads[li] = (d.T @ acts[li], d.sum(axis=0))
        if li > 0:
            d = (d @ W) * gelu_grad(pre[li - 1])
    return np.concatenate([np.concatenate([gW.ravel(), gb]) for gW, gb in grads])


def adam(params, grad, m, v, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (bias-corrected), returns (params, m, v)."""
    m = b1 * m + (1 - b1) * grad
    v = b2 * v + (1 - b2) * grad * grad
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return params - lr * mh / (np.sqrt(vh) + eps), m, v
