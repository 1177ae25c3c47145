"""FP64 reference of the learned row-size predictor.  TEST INFRASTRUCTURE ONLY.

The paper has no such network (it picks one SpGEMM method for the whole
matrix from FLOPs per row, section 2.2.1); this file defines the 3-32-32-1
ReLU regressor plainly so the GPU kernels can be checked against it.

Network, for one row with features x = (log2(1+len), log2(1+ub), log2(1+mx)):
    z1 = W1 x + b1,  h1 = relu(z1)          (32)
    z2 = W2 h1 + b2, h2 = relu(z2)          (32)
    y  = w3 . h2 + b3                        (scalar)
Flat parameter vector (1217 values, row-major): W1[32][3], b1[32],
W2[32][32], b2[32], w3[32], b3.  relu'(0) is taken as 0.
Loss: mean squared error, or the pinball (quantile) loss, over a minibatch.  Optimiser: Adam (Kingma and Ba,
ICLR 2015) with beta1 = 0.9, beta2 = 0.999, eps = 1e-8 and bias correction.

parity unpinned against the paper (no network there); pinned by finite
differences, zero-weight and single-sample closed forms, and loss descent.
"""
from __future__ import annotations

import numpy as np

H = 32
NW = H * 3 + H + H * H + H + H + 1  # 1217

BETA1, BETA2, EPS = 0.9, 0.999, 1e-8


def unpack(w):
    w = np.asarray(w, dtype=np.float64)
    assert w.size == NW
    o = 0
    W1 = w[o:o + H * 3].reshape(H, 3); o += H * 3
    b1 = w[o:o + H]; o += H
    W2 = w[o:o + H * H].reshape(H, H); o += H * H
    b2 = w[o:o + H]; o += H
    w3 = w[o:o + H]; o += H
    b3 = w[o]
    return W1, b1, W2, b2, w3, b3


def pack(W1, b1, W2, b2, w3, b3):
    return np.concatenate([np.ravel(W1), b1, np.ravel(W2), b2, w3, [b3]]).astype(np.float64)


def features(row_len, ub, mx):
    """Row features, FP64: log2 of one plus each count."""
    return np.stack([np.log2(1.0 + np.asarray(row_len, dtype=np.float64)),
                     np.log2(1.0 + np.asarray(ub, dtype=np.float64)),
                     np.log2(1.0 + np.asarray(mx, dtype=np.float64))], axis=1)


def forward(w, X):
    """Returns (y[N], cache) with cache = (X, z1, h1, z2, h2)."""
    W1, b1, W2, b2, w3, b3 = unpack(w)
    X = np.asarray(X, dtype=np.float64)
    z1 = X @ W1.T + b1
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ W2.T + b2
    h2 = np.maximum(z2, 0.0)
    y = h2 @ w3 + b3
    return y, (X, z1, h1, z2, h2)


def backward(w, cache, dy):
    """Gradient of sum_n dy[n] * y[n] with respect to the flat parameters."""
    W1, b1, W2, b2, w3, b3 = unpack(w)
    X, z1, h1, z2, h2 = cache
    dy = np.asarray(dy, dtype=np.float64)
    dw3 = h2.T @ dy
    db3 = dy.sum()
    dz2 = np.outer(dy, w3) * (z2 > 0)
    dW2 = dz2.T @ h1
    db2 = dz2.sum(axis=0)
    dz1 = (dz2 @ W2) * (z1 > 0)
    dW1 = dz1.T @ X
    db1 = dz1.sum(axis=0)
    return pack(dW1, db1, dW2, db2, dw3, db3)


def mse(y, t):
    y = np.asarray(y, dtype=np.float64)
    t = np.asarray(t, dtype=np.float64)
    return float(np.mean((y - t) ** 2)), 2.0 * (y - t) / max(y.size, 1)


def pinball(y, t, q):
    """Pinball loss of level q (mean over rows) and its gradient in y.
    d = t - y; loss q*d for d >= 0, (q-1)*d otherwise; d loss/dy = -q (d > 0),
    1 - q (d <= 0)."""
    y = np.asarray(y, dtype=np.float64)
    t = np.asarray(t, dtype=np.float64)
    d = t - y
    n = max(y.size, 1)
    loss = np.where(d >= 0, q * d, (q - 1.0) * d)
    return float(loss.mean()), np.where(d > 0, -q, 1.0 - q) / n


def adam_step(w, g, m, v, step, lr):
    """One Adam update; ``step`` counts from 1.  Returns new (w, m, v)."""
    m = BETA1 * m + (1.0 - BETA1) * g
    v = BETA2 * v + (1.0 - BETA2) * g * g
    mh = m / (1.0 - BETA1 ** step)
    vh = v / (1.0 - BETA2 ** step)
    return w - lr * mh / (np.sqrt(vh) + EPS), m, v


def train(X, T, w0, epochs, lr, batch, quantile=0.0):
    """Minibatch Adam over the rows in the given order (no reshuffle), on the
    squared error (quantile 0) or the pinball loss of level ``quantile``.

    Returns (w, mean loss per epoch)."""
    w = np.asarray(w0, dtype=np.float64).copy()
    m = np.zeros_like(w)
    v = np.zeros_like(w)
    N = X.shape[0]
    step = 0
    losses = []
    for _ in range(epochs):
        tot = 0.0
        for s in range(0, N, batch):
            xb, tb = X[s:s + batch], T[s:s + batch]
            y, cache = forward(w, xb)
            L, dy = mse(y, tb) if quantile == 0 else pinball(y, tb, quantile)
            g = backward(w, cache, dy)
            step += 1
            w, m, v = adam_step(w, g, m, v, step, lr)
            tot += L * xb.shape[0]
        losses.append(tot / max(N, 1))
    return w, np.asarray(losses)
