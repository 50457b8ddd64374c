"""Float64 reference of the class selector's training math (test infrastructure only).

The network (19 inputs -> 64 ReLU -> 16 scores) and the parameter order are those of the
binary32 selector in pcomp_oracle.c (W1 64x19 row-major, b1, W2 16x64, b2). Training
minimises the mean cross-entropy between softmax(scores) and the class that exhaustive
search picks for each block. This module computes loss and gradients in float64 with plain
numpy, step by step from the definitions (chain rule through the two affine maps, the
ReLU and the softmax); the gradients are pinned against central finite differences.
"""
from __future__ import annotations

import numpy as np

IN, HID, OUT = 19, 64, 16
N_PARAMS = HID * IN + HID + OUT * HID + OUT


def unpack(p):
    p = np.asarray(p, dtype=np.float64)
    o = 0
    W1 = p[o:o + HID * IN].reshape(HID, IN)
    o += HID * IN
    b1 = p[o:o + HID]
    o += HID
    W2 = p[o:o + OUT * HID].reshape(OUT, HID)
    o += OUT * HID
    b2 = p[o:o + OUT]
    return W1, b1, W2, b2


def pack(W1, b1, W2, b2):
    return np.concatenate([W1.reshape(-1), b1, W2.reshape(-1), b2])


def init_params(seed: int) -> np.ndarray:
    """He-style uniform initialisation (float32 values)."""
    rng = np.random.default_rng(seed)
    W1 = rng.uniform(-1, 1, (HID, IN)) * np.sqrt(6.0 / IN)
    W2 = rng.uniform(-1, 1, (OUT, HID)) * np.sqrt(6.0 / HID)
    return pack(W1, np.zeros(HID), W2, np.zeros(OUT)).astype(np.float32)


def forward(p, X):
    """Scores [n, 16] and the hidden pre-activations [n, 64]."""
    W1, b1, W2, b2 = unpack(p)
    X = np.asarray(X, dtype=np.float64)
    A = X @ W1.T + b1
    Hh = np.maximum(A, 0.0)
    S = Hh @ W2.T + b2
    return S, A


def loss(p, X, y) -> float:
    S, _ = forward(p, X)
    S = S - S.max(axis=1, keepdims=True)
    logZ = np.log(np.exp(S).sum(axis=1))
    return float(np.mean(logZ - S[np.arange(len(y)), np.asarray(y, dtype=np.int64)]))


def loss_grad(p, X, y):
    """(mean cross-entropy, gradient in the parameter order)."""
    W1, b1, W2, b2 = unpack(p)
    X = np.asarray(X, dtype=np.float64)
    y = np.asarray(y, dtype=np.int64)
    n = X.shape[0]
    S, A = forward(p, X)
    Hh = np.maximum(A, 0.0)
    Z = S - S.max(axis=1, keepdims=True)
    E = np.exp(Z)
    P = E / E.sum(axis=1, keepdims=True)
    L = float(np.mean(np.log(E.sum(axis=1)) - Z[np.arange(n), y]))
    dS = P.copy()
    dS[np.arange(n), y] -= 1.0
    dS /= n
    gW2 = dS.T @ Hh
    gb2 = dS.sum(axis=0)
    dH = dS @ W2
    dA = dH * (A > 0.0)
    gW1 = dA.T @ X
    gb1 = dA.sum(axis=0)
    return L, pack(gW1, gb1, gW2, gb2)


def adam_step(p, g, m, v, t: int, lr: float, b1: float = 0.9, b2: float = 0.999, eps: float = 1e-8):
    """One Adam update (Kingma & Ba, 2015, Algorithm 1), t counted from 1."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v
