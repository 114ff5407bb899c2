"""Float64 reference of the cost-model MLP (test infrastructure).

    h1 = relu(x W1 + b1)      x: [B, F], W1: [F, H]
    h2 = relu(h1 W2 + b2)     W2: [H, H]
    y  = h2 w3 + b3           w3: [H]
    L  = mean_b (y_b - t_b)^2

Gradients by the chain rule written out layer by layer; pinned in the tests
by central finite differences.  Parameter vector order (the library's):
W1 (row-major F x H), b1, W2 (row-major H x H), b2, w3, b3.
"""
from __future__ import annotations

import numpy as np


def unpack(theta, F, H):
    i = 0
    W1 = theta[i:i + F * H].reshape(F, H); i += F * H
    b1 = theta[i:i + H]; i += H
    W2 = theta[i:i + H * H].reshape(H, H); i += H * H
    b2 = theta[i:i + H]; i += H
    w3 = theta[i:i + H]; i += H
    b3 = theta[i]; i += 1
    assert i == len(theta)
    return W1, b1, W2, b2, w3, b3


def num_params(F, H):
    return F * H + H + H * H + H + H + 1


def forward(theta, X, F, H):
    W1, b1, W2, b2, w3, b3 = unpack(np.asarray(theta, np.float64), F, H)
    X = np.asarray(X, np.float64)
    z1 = X @ W1 + b1
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ W2 + b2
    h2 = np.maximum(z2, 0.0)
    y = h2 @ w3 + b3
    return y, (X, z1, h1, z2, h2)


def loss(theta, X, t, F, H):
    y, _ = forward(theta, X, F, H)
    return float(np.mean((y - np.asarray(t, np.float64)) ** 2))


def gradients(theta, X, t, F, H):
    W1, b1, W2, b2, w3, b3 = unpack(np.asarray(theta, np.float64), F, H)
    y, (X, z1, h1, z2, h2) = forward(theta, X, F, H)
    B = X.shape[0]
    dy = 2.0 * (y - np.asarray(t, np.float64)) / B          # dL/dy
    dw3 = h2.T @ dy
    db3 = dy.sum()
    dz2 = np.outer(dy, w3) * (z2 > 0)
    dW2 = h1.T @ dz2
    db2 = dz2.sum(axis=0)
    dz1 = (dz2 @ W2.T) * (z1 > 0)
    dW1 = X.T @ dz1
    db1 = dz1.sum(axis=0)
    return np.concatenate([dW1.ravel(), db1, dW2.ravel(), db2, dw3, [db3]])
