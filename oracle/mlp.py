"""Leaf-proposal MLP (oracle, FP64).  Test infra only.

A small network maps a PCA-reduced query q' to scores over the leaves of the
k-means search tree, so that a query can be sent straight to its most likely
leaves instead of descending the tree.  Shapes n_in -> h -> h -> n_out
(64 -> 256 -> 256 -> 1024 in the learned workload), GELU with the exact
error function, GELU(x) = x * Phi(x).

Definitions:
  a0 = q' * s           (s = fixed per-feature input scale, not trained)
  h1 = GELU(W1 a0 + b1), h2 = GELU(W2 h1 + b2), logits = W3 h2 + b3
  loss = mean over the batch of logsumexp(logits) - logits[label]
  proposal = the 4 largest logits (ties to the lowest leaf),
  margin = p_(1) - p_(2) of softmax(logits).
  Adam (Kingma & Ba): m = b1 m + (1-b1) g; v = b2 v + (1-b2) g^2;
  theta -= lr * (m / (1-b1^t)) / (sqrt(v / (1-b2^t)) + eps).

Parameters are packed as W1 [h][n_in], b1 [h], W2 [h][h], b2 [h],
W3 [n_out][h], b3 [n_out], row-major, in that order.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf


def shapes(n_in: int, h: int, n_out: int):
    return [(h, n_in), (h,), (h, h), (h,), (n_out, h), (n_out,)]


def n_params(n_in: int, h: int, n_out: int) -> int:
    return sum(int(np.prod(s)) for s in shapes(n_in, h, n_out))


def unpack(theta: np.ndarray, n_in: int, h: int, n_out: int):
    out, o = [], 0
    for s in shapes(n_in, h, n_out):
        k = int(np.prod(s))
        out.append(np.asarray(theta[o : o + k], dtype=np.float64).reshape(s))
        o += k
    return out


def pack(parts) -> np.ndarray:
    return np.concatenate([np.asarray(p, dtype=np.float64).reshape(-1) for p in parts])


def gelu(x):
    return x * 0.5 * (1.0 + erf(x / math.sqrt(2.0)))


def gelu_grad(x):
    return 0.5 * (1.0 + erf(x / math.sqrt(2.0))) + x * np.exp(-0.5 * x * x) / math.sqrt(2.0 * math.pi)


def forward(theta, q, n_in, h, n_out, in_scale=None):
    W1, b1, W2, b2, W3, b3 = unpack(theta, n_in, h, n_out)
    a0 = np.asarray(q, dtype=np.float64)
    if in_scale is not None:
        a0 = a0 * np.asarray(in_scale, dtype=np.float64)[None, :]
    z1 = a0 @ W1.T + b1
    h1 = gelu(z1)
    z2 = h1 @ W2.T + b2
    h2 = gelu(z2)
    logits = h2 @ W3.T + b3
    return logits, (a0, z1, h1, z2, h2)


def loss_and_grad(theta, q, labels, n_in, h, n_out, in_scale=None):
    """Mean softmax cross-entropy and its gradient (packed like theta)."""
    W1, b1, W2, b2, W3, b3 = unpack(theta, n_in, h, n_out)
    logits, (a0, z1, h1, z2, h2) = forward(theta, q, n_in, h, n_out, in_scale)
    n = logits.shape[0]
    labels = np.asarray(labels, dtype=np.int64)
    m = logits.max(axis=1, keepdims=True)
    e = np.exp(logits - m)
    Zs = e.sum(axis=1, keepdims=True)
    lse = (m + np.log(Zs))[:, 0]
    loss = float(np.mean(lse - logits[np.arange(n), labels]))
    g = e / Zs
    g[np.arange(n), labels] -= 1.0
    g /= n
    dW3 = g.T @ h2
    db3 = g.sum(axis=0)
    dz2 = (g @ W3) * gelu_grad(z2)
    dW2 = dz2.T @ h1
    db2 = dz2.sum(axis=0)
    dz1 = (dz2 @ W2) * gelu_grad(z1)
    dW1 = dz1.T @ a0
    db1 = dz1.sum(axis=0)
    return loss, pack([dW1, db1, dW2, db2, dW3, db3])


def loss_only(theta, q, labels, n_in, h, n_out, in_scale=None) -> float:
    logits, _ = forward(theta, q, n_in, h, n_out, in_scale)
    m = logits.max(axis=1, keepdims=True)
    lse = (m + np.log(np.exp(logits - m).sum(axis=1, keepdims=True)))[:, 0]
    labels = np.asarray(labels, dtype=np.int64)
    return float(np.mean(lse - logits[np.arange(logits.shape[0]), labels]))


def adam_step(theta, grad, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update at step t (1-based); returns (theta, m, v)."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mh = m / (1.0 - beta1**t)
    vh = v / (1.0 - beta2**t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def propose(logits, k: int = 4):
    """Top-k leaves (ties to the lowest index) and softmax margin p1 - p2."""
    logits = np.asarray(logits, dtype=np.float64)
    n, L = logits.shape
    order = np.lexsort((np.broadcast_to(np.arange(L), logits.shape), -logits), axis=1)[:, :k]
    top = np.take_along_axis(logits, order, axis=1)
    Zs = np.exp(logits - top[:, :1]).sum(axis=1)
    p1 = 1.0 / Zs
    p2 = np.exp(top[:, 1] - top[:, 0]) / Zs if k > 1 else np.zeros(n)
    return order, p1 - p2
