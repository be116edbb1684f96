"""Float64 reference of the scorer's training loss and gradient.

TEST INFRASTRUCTURE ONLY (CPU oracle; shares no code with the HIP path).
Network: h1 = relu(W1 x + b1), h2 = relu(W2 h1 + b2), z = W3 h2 + b3; loss
is the softmax cross-entropy restricted to the feasible types (mask bits),
averaged over the minibatch.  Parameters are taken at their bf16 values.
"""
from __future__ import annotations

import numpy as np


def unpack(flat: np.ndarray, n_out: int):
    o = 0
    def take(k, shape=None):
        nonlocal o
        v = flat[o:o + k]
        o += k
        return v.reshape(shape) if shape else v
    w1 = take(1024, (64, 16)); b1 = take(64)
    w2 = take(4096, (64, 64)); b2 = take(64)
    w3 = take(64 * n_out, (n_out, 64)); b3 = take(n_out)
    return w1, b1, w2, b2, w3, b3


def loss_and_grad(flat, n_out, X, mask, label):
    """Mean masked cross-entropy and its gradient (float64)."""
    w1, b1, w2, b2, w3, b3 = unpack(np.asarray(flat, np.float64), n_out)
    X = np.asarray(X, np.float64)
    B = X.shape[0]
    a1 = X @ w1.T + b1
    h1 = np.maximum(a1, 0)
    a2 = h1 @ w2.T + b2
    h2 = np.maximum(a2, 0)
    z = h2 @ w3.T + b3
    feas = ((np.asarray(mask, np.int64)[:, None] >> np.arange(n_out)) & 1).astype(bool)
    zm = np.where(feas, z, -np.inf)
    zmax = zm.max(1, keepdims=True)
    e = np.where(feas, np.exp(zm - zmax), 0.0)
    s = e.sum(1, keepdims=True)
    p = e / s
    lab = np.asarray(label, np.int64)
    loss = float(np.mean(-(z[np.arange(B), lab] - zmax[:, 0] - np.log(s[:, 0]))))
    dz = p.copy()
    dz[np.arange(B), lab] -= 1.0
    dz /= B
    gw3 = dz.T @ h2
    gb3 = dz.sum(0)
    dh2 = (dz @ w3) * (a2 > 0)
    gw2 = dh2.T @ h1
    gb2 = dh2.sum(0)
    dh1 = (dh2 @ w2) * (a1 > 0)
    gw1 = dh1.T @ X
    gb1 = dh1.sum(0)
    grad = np.concatenate([gw1.ravel(), gb1, gw2.ravel(), gb2, gw3.ravel(), gb3])
    return loss, grad


def loss_only(flat, n_out, X, mask, label):
    return loss_and_grad(flat, n_out, X, mask, label)[0]
