"""Plain FP64 reference of the signed-distance surrogate network.

TEST INFRASTRUCTURE ONLY: only the tests, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this module.

Network (the learned-indicator workload; not part of the paper, whose hook is
Sec. 5.4: non-spherical signed distances are costlier per lattice node):
    h1 = silu(W1 x + b1)        3 -> 64
    h2 = silu(W2 h1 + b2)       64 -> 64
    h3 = silu(W3 h2 + b3)       64 -> 64
    y  = W4 . h3 + b4           64 -> 1
with silu(z) = z / (1 + exp(-z)), loss L = mean_s (y_s - t_s)^2, and Adam.

Parameters are one flat FP32/FP64 vector of 8641 entries in the order
W1 (64x3, row-major), b1, W2 (64x64), b2, W3 (64x64), b3, W4 (64), b4.

``bf16=True`` rounds, to bfloat16 with round-to-nearest-even, exactly the
operands a BF16 matrix-core implementation feeds its two 64x64 products:
the weights W2, W3, the layer inputs h1, h2 in the forward pass and the
back-propagated errors d3, d2 in the backward pass.  Everything else,
including every sum, stays FP64.
"""
from __future__ import annotations

import numpy as np

H = 64
SIZES = [("W1", (H, 3)), ("b1", (H,)), ("W2", (H, H)), ("b2", (H,)), ("W3", (H, H)),
         ("b3", (H,)), ("W4", (H,)), ("b4", (1,))]
NPARAM = sum(int(np.prod(s)) for _, s in SIZES)


def unpack(theta):
    out, k = {}, 0
    for name, shp in SIZES:
        n = int(np.prod(shp))
        out[name] = np.asarray(theta[k:k + n], dtype=np.float64).reshape(shp)
        k += n
    return out


def pack(p):
    return np.concatenate([np.asarray(p[name], dtype=np.float64).reshape(-1) for name, _ in SIZES])


def bf16_round(a):
    """Round to the nearest bfloat16 (ties to even), returned as float64."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000).astype(np.uint32)
    return r.view(np.float32).astype(np.float64)


def silu(z):
    return z / (1.0 + np.exp(-z))


def dsilu(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def forward(theta, X, bf16=False):
    """y[n] for inputs X[n, 3]; also returns the intermediate values."""
    p = unpack(theta)
    rnd = bf16_round if bf16 else (lambda a: a)
    X = np.asarray(X, dtype=np.float64)
    z1 = X @ p["W1"].T + p["b1"]
    h1 = silu(z1)
    z2 = rnd(h1) @ rnd(p["W2"]).T + p["b2"]
    h2 = silu(z2)
    z3 = rnd(h2) @ rnd(p["W3"]).T + p["b3"]
    h3 = silu(z3)
    y = h3 @ p["W4"] + p["b4"][0]
    return y, dict(z1=z1, h1=h1, z2=z2, h2=h2, z3=z3, h3=h3)


def loss(theta, X, t, bf16=False):
    y, _ = forward(theta, X, bf16)
    return float(np.mean((y - t) ** 2))


def gradient(theta, X, t, bf16=False):
    """Gradient of the mean-squared loss by back-propagation; returns (grad, loss)."""
    p = unpack(theta)
    rnd = bf16_round if bf16 else (lambda a: a)
    X = np.asarray(X, dtype=np.float64)
    t = np.asarray(t, dtype=np.float64)
    y, c = forward(theta, X, bf16)
    n = len(X)
    dy = 2.0 * (y - t) / n
    g = {}
    g["W4"] = c["h3"].T @ dy
    g["b4"] = np.array([dy.sum()])
    d3 = (dy[:, None] * p["W4"][None, :]) * dsilu(c["z3"])
    g["W3"] = rnd(d3).T @ rnd(c["h2"])
    g["b3"] = d3.sum(0)
    d2 = (rnd(d3) @ rnd(p["W3"])) * dsilu(c["z2"])
    g["W2"] = rnd(d2).T @ rnd(c["h1"])
    g["b2"] = d2.sum(0)
    d1 = (rnd(d2) @ rnd(p["W2"])) * dsilu(c["z1"])
    g["W1"] = d1.T @ X
    g["b1"] = d1.sum(0)
    return pack(g), float(np.mean((y - t) ** 2))


def adam_step(theta, m, v, grad, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba 2015) with bias correction; step >= 1."""
    m = beta1 * m + (1 - beta1) * grad
    v = beta2 * v + (1 - beta2) * grad * grad
    mhat = m / (1 - beta1 ** step)
    vhat = v / (1 - beta2 ** step)
    return theta - lr * mhat / (np.sqrt(vhat) + eps), m, v
