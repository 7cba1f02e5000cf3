"""FP64 numpy reference of the surrogate network -- TEST INFRASTRUCTURE.

A plain multilayer perceptron y = L_n(s(L_{n-1}(... s(L_1(x))))) with
L_l(h) = h W_l^T + b_l (W_l stored [out, in]), SiLU s(z) = z / (1 + e^-z)
on every hidden layer and a linear output; mean-squared-error loss; Adam.
It is the reference the library's training kernels are checked against and
shares no code with them.  Parameters are packed as W_1, b_1, W_2, b_2, ...
(row-major), the layout the library's C interface uses.
"""
from __future__ import annotations

import numpy as np


def shapes(widths):
    return [((widths[l + 1], widths[l]), (widths[l + 1],)) for l in range(len(widths) - 1)]


def num_params(widths) -> int:
    return sum(o * i + o for (o, i), _ in shapes(widths))


def unpack(theta, widths):
    out, p = [], 0
    for (o, i), _ in shapes(widths):
        W = theta[p:p + o * i].reshape(o, i); p += o * i
        b = theta[p:p + o]; p += o
        out.append((W, b))
    return out


def pack(layers):
    return np.concatenate([np.concatenate([W.ravel(), b.ravel()]) for W, b in layers])


def he_uniform(widths, seed: int):
    """W ~ U(-sqrt(6/fan_in), +sqrt(6/fan_in)), b = 0."""
    rng = np.random.default_rng(seed)
    layers = []
    for (o, i), _ in shapes(widths):
        lim = np.sqrt(6.0 / i)
        layers.append((rng.uniform(-lim, lim, (o, i)), np.zeros(o)))
    return pack(layers)


def silu(z):
    return z / (1.0 + np.exp(-z))


def silu_grad(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def forward(theta, widths, x):
    """Returns the output and the per-layer (input, pre-activation) cache."""
    h = np.asarray(x, dtype=np.float64)
    cache = []
    layers = unpack(np.asarray(theta, dtype=np.float64), widths)
    for l, (W, b) in enumerate(layers):
        z = h @ W.T + b
        cache.append((h, z))
        h = silu(z) if l < len(layers) - 1 else z
    return h, cache


def mse(y, t):
    """loss = mean((y - t)^2), dloss/dy."""
    d = np.asarray(y, np.float64) - np.asarray(t, np.float64)
    return float(np.mean(d * d)), 2.0 * d / d.size


def backward(theta, widths, cache, dy):
    """Gradient of a scalar with d/dy = dy, packed like theta."""
    layers = unpack(np.asarray(theta, dtype=np.float64), widths)
    grads = [None] * len(layers)
    g = np.asarray(dy, dtype=np.float64)
    for l in range(len(layers) - 1, -1, -1):
        W, _ = layers[l]
        h, z = cache[l]
        if l < len(layers) - 1:
            g = g * silu_grad(z)
        grads[l] = (g.T @ h, g.sum(axis=0))
        g = g @ W
    return pack(grads)


def adam(theta, grad, m, v, step: int, lr: float, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step (bias-corrected moments); returns new theta, m, v."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mh = m / (1.0 - beta1 ** step)
    vh = v / (1.0 - beta2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v
