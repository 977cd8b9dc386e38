"""FP64 numpy oracle of the precision-selector MLP — TEST INFRASTRUCTURE ONLY.

Network: 16 -> 64 -> 64 -> 3, ReLU on the hidden layers, softmax output,
mean cross-entropy loss; Adam update (Kingma & Ba 2015, Algorithm 1).
Parameter blob layout (float, contiguous, 5443 values):
  W1 (64 x 16, row-major: W1[o, i]), b1 (64), W2 (64 x 64), b2 (64),
  W3 (3 x 64), b3 (3).
"""
from __future__ import annotations

import numpy as np

SIZES = [(64, 16), (64,), (64, 64), (64,), (3, 64), (3,)]
NPARAM = sum(int(np.prod(s)) for s in SIZES)  # 5443


def unpack(theta):
    theta = np.asarray(theta, dtype=np.float64)
    out, o = [], 0
    for s in SIZES:
        k = int(np.prod(s))
        out.append(theta[o:o + k].reshape(s))
        o += k
    return out


def pack(parts):
    return np.concatenate([np.asarray(p, dtype=np.float64).ravel() for p in parts])


def forward(theta, X):
    """Returns (probabilities N x 3, cache)."""
    W1, b1, W2, b2, W3, b3 = unpack(theta)
    X = np.asarray(X, dtype=np.float64)
    z1 = X @ W1.T + b1
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ W2.T + b2
    h2 = np.maximum(z2, 0.0)
    z3 = h2 @ W3.T + b3
    z3s = z3 - z3.max(axis=1, keepdims=True)
    e = np.exp(z3s)
    p = e / e.sum(axis=1, keepdims=True)
    return p, (X, z1, h1, z2, h2, z3)


def loss(theta, X, y):
    p, _ = forward(theta, X)
    y = np.asarray(y)
    return float(-np.mean(np.log(p[np.arange(len(y)), y])))


def backward(theta, X, y):
    """Analytic gradient of the mean cross-entropy w.r.t. theta."""
    W1, b1, W2, b2, W3, b3 = unpack(theta)
    p, (X, z1, h1, z2, h2, z3) = forward(theta, X)
    N = X.shape[0]
    y = np.asarray(y)
    g3 = p.copy()
    g3[np.arange(N), y] -= 1.0
    g3 /= N
    dW3 = g3.T @ h2
    db3 = g3.sum(axis=0)
    g2 = (g3 @ W3) * (z2 > 0)
    dW2 = g2.T @ h1
    db2 = g2.sum(axis=0)
    g1 = (g2 @ W2) * (z1 > 0)
    dW1 = g1.T @ X
    db1 = g1.sum(axis=0)
    return pack([dW1, db1, dW2, db2, dW3, db3])


def adam_step(theta, grad, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (t is the 1-based step count). Returns (theta, m, v)."""
    m = b1 * m + (1.0 - b1) * grad
    v = b2 * v + (1.0 - b2) * grad * grad
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    theta = theta - lr * mh / (np.sqrt(vh) + eps)
    return theta, m, v
