"""CPU float64 reference of the work predictor (test infrastructure only).

The network maps F = 10 item features through two hidden layers of 32 ReLU
units to one linear output; the loss is 0.5 * mean over samples of
(prediction - target)^2.  Parameters are one flat vector: W1 (32 x F, row =
output unit), b1 (32), W2 (32 x 32), b2 (32), W3 (32), b3 (1) -- the layout
the GPU library exposes, so that both sides can be handed the same vector.

Backward is the chain rule written out layer by layer; it is pinned by
central finite differences of the loss (tests/test_mlp_oracle.py).
"""
from __future__ import annotations

import numpy as np

F = 10
HID = 32
SIZES = [("W1", (HID, F)), ("b1", (HID,)), ("W2", (HID, HID)), ("b2", (HID,)), ("W3", (HID,)), ("b3", (1,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SIZES)


def unpack(p):
    p = np.asarray(p, dtype=np.float64)
    assert p.shape == (N_PARAMS,)
    out, off = {}, 0
    for name, shape in SIZES:
        k = int(np.prod(shape))
        out[name] = p[off:off + k].reshape(shape)
        off += k
    return out


def pack(d):
    return np.concatenate([np.asarray(d[name], dtype=np.float64).reshape(-1) for name, _ in SIZES])


def forward(p, X):
    """Predictions for the rows of X (n x F) and the hidden activations."""
    w = unpack(p)
    X = np.asarray(X, dtype=np.float64)
    z1 = X @ w["W1"].T + w["b1"]
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ w["W2"].T + w["b2"]
    h2 = np.maximum(z2, 0.0)
    y = h2 @ w["W3"] + w["b3"][0]
    return y, (X, z1, h1, z2, h2)


def loss(p, X, t):
    y, _ = forward(p, X)
    r = y - np.asarray(t, dtype=np.float64)
    return 0.5 * float(np.mean(r * r))


def loss_grad(p, X, t):
    """Loss and its gradient with respect to the flat parameter vector."""
    w = unpack(p)
    y, (X, z1, h1, z2, h2) = forward(p, X)
    n = X.shape[0]
    r = y - np.asarray(t, dtype=np.float64)
    L = 0.5 * float(np.mean(r * r))
    gy = r / n                                  # dL/dy per sample
    g = {"W3": h2.T @ gy, "b3": np.array([gy.sum()])}
    gz2 = np.outer(gy, w["W3"]) * (z2 > 0)      # dL/dz2
    g["W2"] = gz2.T @ h1
    g["b2"] = gz2.sum(axis=0)
    gz1 = (gz2 @ w["W2"]) * (z1 > 0)            # dL/dz1
    g["W1"] = gz1.T @ X
    g["b1"] = gz1.sum(axis=0)
    return L, pack(g)


def finite_diff(p, X, t, idx, h=1e-6):
    """Central differences of the loss for the parameters listed in idx."""
    p = np.asarray(p, dtype=np.float64).copy()
    out = np.zeros(len(idx))
    for k, i in enumerate(idx):
        old = p[i]
        p[i] = old + h
        lp = loss(p, X, t)
        p[i] = old - h
        lm = loss(p, X, t)
        p[i] = old
        out[k] = (lp - lm) / (2 * h)
    return out
