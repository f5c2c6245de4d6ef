"""FP64 reference of the schedule cost model's network and its training step.

Test infrastructure only (tests, smoke check and the benchmark's CPU leg):
nothing in the product imports this module.

The network maps standardised features x' = (x - mean) * inv_std to a
predicted log run time through two hidden layers of 64 ReLU units:

    h1 = relu(W1 x' + b1),  h2 = relu(W2 h1 + b2),  y = w3 . h2 + b3.

Training minimises L = mean_s (y_s - t_s)^2 with Adam (Kingma and Ba, 2015):
    m <- b1 m + (1 - b1) g,  v <- b2 v + (1 - b2) g^2,
    p <- p - lr * (m / (1 - b1^k)) / (sqrt(v / (1 - b2^k)) + eps)
at update k = 1, 2, ...  The flat parameter order is W1 (64 x in, row-major),
b1, W2 (64 x 64), b2, w3, b3. The derivative of relu at 0 is taken as 0.

Pins (tests/test_mlp_oracle.py): central finite differences of L, a network
small enough to evaluate by hand, the first Adam step's closed form, and the
scalar Adam recurrence written out for two steps.
"""
from __future__ import annotations

import numpy as np

HIDDEN = 64


def layout(in_dim: int) -> dict:
    h = HIDDEN
    o = {}
    o["W1"] = (0, (h, in_dim))
    o["b1"] = (h * in_dim, (h,))
    o["W2"] = (h * in_dim + h, (h, h))
    o["b2"] = (h * in_dim + h + h * h, (h,))
    o["w3"] = (h * in_dim + 2 * h + h * h, (h,))
    o["b3"] = (h * in_dim + 3 * h + h * h, ())
    return o


def param_count(in_dim: int) -> int:
    return HIDDEN * in_dim + 3 * HIDDEN + HIDDEN * HIDDEN + 1


def unpack(params: np.ndarray, in_dim: int) -> dict:
    p = np.asarray(params, dtype=np.float64)
    assert p.size == param_count(in_dim)
    out = {}
    for name, (off, shape) in layout(in_dim).items():
        size = int(np.prod(shape)) if shape else 1
        out[name] = p[off:off + size].reshape(shape) if shape else p[off]
    return out


def pack(t: dict, in_dim: int) -> np.ndarray:
    p = np.zeros(param_count(in_dim))
    for name, (off, shape) in layout(in_dim).items():
        v = np.asarray(t[name], dtype=np.float64).reshape(-1)
        p[off:off + v.size] = v
    return p


def standardise(x: np.ndarray, norm) -> np.ndarray:
    x = np.asarray(x, dtype=np.float64)
    if norm is None:
        return x
    norm = np.asarray(norm, dtype=np.float64)
    d = x.shape[1]
    return (x - norm[:d]) * norm[d:]


def forward(params, norm, x) -> np.ndarray:
    """Predictions for every row of x (batch x in)."""
    x = np.atleast_2d(np.asarray(x, dtype=np.float64))
    t = unpack(params, x.shape[1])
    xs = standardise(x, norm)
    h1 = np.maximum(xs @ t["W1"].T + t["b1"], 0.0)
    h2 = np.maximum(h1 @ t["W2"].T + t["b2"], 0.0)
    return h2 @ t["w3"] + t["b3"]


def loss(params, norm, x, target) -> float:
    y = forward(params, norm, x)
    return float(np.mean((y - np.asarray(target, dtype=np.float64)) ** 2))


def loss_and_grad(params, norm, x, target):
    """(L, dL/dparams) by the chain rule, layer by layer."""
    x = np.atleast_2d(np.asarray(x, dtype=np.float64))
    target = np.asarray(target, dtype=np.float64)
    d = x.shape[1]
    t = unpack(params, d)
    b = x.shape[0]
    xs = standardise(x, norm)
    z1 = xs @ t["W1"].T + t["b1"]
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ t["W2"].T + t["b2"]
    h2 = np.maximum(z2, 0.0)
    y = h2 @ t["w3"] + t["b3"]
    r = y - target
    L = float(np.mean(r * r))
    dy = 2.0 * r / b                       # dL/dy_s
    g = {}
    g["w3"] = h2.T @ dy
    g["b3"] = np.sum(dy)
    dz2 = np.outer(dy, t["w3"]) * (z2 > 0)
    g["W2"] = dz2.T @ h1
    g["b2"] = np.sum(dz2, axis=0)
    dz1 = (dz2 @ t["W2"]) * (z1 > 0)
    g["W1"] = dz1.T @ xs
    g["b1"] = np.sum(dz1, axis=0)
    return L, pack(g, d)


def adam_step(params, m, v, grad, lr, beta1, beta2, eps, step):
    """One bias-corrected Adam update; returns new (params, m, v)."""
    params = np.asarray(params, dtype=np.float64)
    grad = np.asarray(grad, dtype=np.float64)
    m = beta1 * np.asarray(m, dtype=np.float64) + (1.0 - beta1) * grad
    v = beta2 * np.asarray(v, dtype=np.float64) + (1.0 - beta2) * grad * grad
    mh = m / (1.0 - beta1 ** step)
    vh = v / (1.0 - beta2 ** step)
    return params - lr * mh / (np.sqrt(vh) + eps), m, v
