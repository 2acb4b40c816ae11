"""FP64 reference of the block screener's network (test infrastructure only).

A 3-layer perceptron  x (F) -> 64 -> 64 -> 1  with ReLU activations:
    h1 = relu(W1 x + b1),  h2 = relu(W2 h1 + b2),  y = W3 h2 + b3
trained with an asymmetric squared loss on r = y - t (t the target log10 norm),
    L = (1/n) sum_i w(r_i) r_i^2,   w = 1 if r >= 0 else alpha,
which penalises under-prediction (a block predicted smaller than it is could be
skipped wrongly), and the Adam update (Kingma & Ba, ICLR 2015):
    m = b1 m + (1-b1) g,  v = b2 v + (1-b2) g^2,
    p -= lr * (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).

Pinned by: gradients against central finite differences of the loss
(tests/test_oracle_mlp.py); the GPU kernels are then checked against this module.
"""
from __future__ import annotations

import numpy as np

NAMES = ("w1", "b1", "w2", "b2", "w3", "b3")


def init(n_in, hidden=64, seed=0):
    rng = np.random.default_rng(seed)
    p = {
        "w1": rng.standard_normal((hidden, n_in)) * np.sqrt(2.0 / n_in),
        "b1": np.zeros(hidden),
        "w2": rng.standard_normal((hidden, hidden)) * np.sqrt(2.0 / hidden),
        "b2": np.zeros(hidden),
        "w3": rng.standard_normal((1, hidden)) * np.sqrt(1.0 / hidden),
        "b3": np.zeros(1),
    }
    return p


def forward(p, x):
    a1 = x @ p["w1"].T + p["b1"]
    h1 = np.maximum(a1, 0.0)
    a2 = h1 @ p["w2"].T + p["b2"]
    h2 = np.maximum(a2, 0.0)
    y = (h2 @ p["w3"].T + p["b3"])[:, 0]
    return y, (x, a1, h1, a2, h2)


def loss(p, x, t, alpha):
    y, _ = forward(p, x)
    r = y - t
    w = np.where(r >= 0, 1.0, alpha)
    return float(np.mean(w * r * r))


def backward(p, x, t, alpha):
    """Loss and gradients of every parameter."""
    y, (x, a1, h1, a2, h2) = forward(p, x)
    n = x.shape[0]
    r = y - t
    w = np.where(r >= 0, 1.0, alpha)
    dy = 2.0 * w * r / n                       # dL/dy
    g = {}
    g["w3"] = dy[None, :] @ h2
    g["b3"] = np.array([dy.sum()])
    dh2 = dy[:, None] * p["w3"]                # [n, H]
    da2 = dh2 * (a2 > 0)
    g["w2"] = da2.T @ h1
    g["b2"] = da2.sum(0)
    dh1 = da2 @ p["w2"]
    da1 = dh1 * (a1 > 0)
    g["w1"] = da1.T @ x
    g["b1"] = da1.sum(0)
    return float(np.mean(w * r * r)), g


def adam(p, g, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    for k in NAMES:
        m[k] = beta1 * m[k] + (1 - beta1) * g[k]
        v[k] = beta2 * v[k] + (1 - beta2) * g[k] * g[k]
        mh = m[k] / (1 - beta1 ** step)
        vh = v[k] / (1 - beta2 ** step)
        p[k] = p[k] - lr * mh / (np.sqrt(vh) + eps)
    return p, m, v
