"""fp64 reference of the cost-model network (test infrastructure only).

The network maps a 16-value feature vector to one prediction:
    h1 = relu(W1 x + b1), h2 = relu(W2 h1 + b2), y = W3 h2 + b3,
trained on the mean squared error L = mean_s (y_s - t_s)^2 with Adam
(Kingma & Ba, 2015).  Parameters are one flat array laid out as
W1[H][16], b1[H], W2[H][H], b2[H], W3[H], b3.

The gradient below is written from the chain rule, term by term; the tests
pin it with central finite differences and closed forms.
"""
from __future__ import annotations

import numpy as np

N_IN = 16


def param_count(h: int) -> int:
    return h * N_IN + h + h * h + h + h + 1


def unpack(p: np.ndarray, h: int):
    p = np.asarray(p, np.float64)
    o = 0
    W1 = p[o:o + h * N_IN].reshape(h, N_IN); o += h * N_IN
    b1 = p[o:o + h]; o += h
    W2 = p[o:o + h * h].reshape(h, h); o += h * h
    b2 = p[o:o + h]; o += h
    W3 = p[o:o + h]; o += h
    b3 = p[o]
    return W1, b1, W2, b2, W3, b3


def forward(p, x, h):
    W1, b1, W2, b2, W3, b3 = unpack(p, h)
    x = np.asarray(x, np.float64)
    a1 = np.maximum(x @ W1.T + b1, 0.0)
    a2 = np.maximum(a1 @ W2.T + b2, 0.0)
    return a2 @ W3 + b3


def loss_grad(p, x, t, h):
    """Mean squared error and its gradient with respect to every parameter."""
    W1, b1, W2, b2, W3, b3 = unpack(p, h)
    x = np.asarray(x, np.float64)
    t = np.asarray(t, np.float64)
    n = len(t)
    z1 = x @ W1.T + b1
    a1 = np.maximum(z1, 0.0)
    z2 = a1 @ W2.T + b2
    a2 = np.maximum(z2, 0.0)
    y = a2 @ W3 + b3
    e = y - t
    loss = float(np.mean(e * e))
    dy = 2.0 * e / n                      # dL/dy_s
    dW3 = a2.T @ dy
    db3 = dy.sum()
    dz2 = np.outer(dy, W3) * (z2 > 0)     # dL/dz2
    dW2 = dz2.T @ a1
    db2 = dz2.sum(axis=0)
    dz1 = (dz2 @ W2) * (z1 > 0)
    dW1 = dz1.T @ x
    db1 = dz1.sum(axis=0)
    g = np.concatenate([dW1.ravel(), db1, dW2.ravel(), db2, dW3, [db3]])
    return loss, g


def adam(p, g, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


def init(h: int, seed: int = 0) -> np.ndarray:
    """He-style random initialisation (deterministic for a seed)."""
    rng = np.random.default_rng(seed)
    parts = [rng.normal(0, np.sqrt(2.0 / N_IN), h * N_IN), np.zeros(h),
             rng.normal(0, np.sqrt(2.0 / h), h * h), np.zeros(h),
             rng.normal(0, np.sqrt(1.0 / h), h), np.zeros(1)]
    return np.concatenate(parts)
