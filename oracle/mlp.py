"""The bound-predictor network in FP64: 9 -> 64 -> 64 -> 64 -> 3, tanh hidden
layers, linear output, with its exact gradient and one Adam update.

Packed parameter layout (shared convention of the C-ABI, float32 on the GPU):
for each layer l = 1..4 in order, W_l as [in][out] row-major, then b_l[out].
Activation cache layout: X [B][9] | H1 [B][64] | H2 [B][64] | H3 [B][64].

Adam (Kingma & Ba 2015, Algorithm 1): m <- b1 m + (1-b1) g,
v <- b2 v + (1-b2) g^2, W <- W - lr (m / (1-b1^t)) / (sqrt(v / (1-b2^t)) + eps).
"""
from __future__ import annotations

import numpy as np

SIZES = (9, 64, 64, 64, 3)


def n_params(sizes=SIZES) -> int:
    return sum(a * b + b for a, b in zip(sizes[:-1], sizes[1:]))


def unpack(W, sizes=SIZES):
    out = []
    o = 0
    for a, b in zip(sizes[:-1], sizes[1:]):
        Wl = np.asarray(W[o:o + a * b], dtype=np.float64).reshape(a, b)
        o += a * b
        bl = np.asarray(W[o:o + b], dtype=np.float64)
        o += b
        out.append((Wl, bl))
    return out


def pack(layers) -> np.ndarray:
    return np.concatenate([np.concatenate([Wl.ravel(), bl.ravel()]) for Wl, bl in layers])


def init_params(seed: int, sizes=SIZES) -> np.ndarray:
    """Glorot-uniform weights, zero biases (seeded)."""
    rng = np.random.default_rng(seed)
    layers = []
    for a, b in zip(sizes[:-1], sizes[1:]):
        lim = np.sqrt(6.0 / (a + b))
        layers.append((rng.uniform(-lim, lim, size=(a, b)), np.zeros(b)))
    return pack(layers)


def forward(W, X):
    """Returns (Y, cache); cache = [X, H1, H2, H3]."""
    layers = unpack(W)
    H = np.asarray(X, dtype=np.float64)
    cache = [H]
    for i, (Wl, bl) in enumerate(layers):
        Z = H @ Wl + bl
        if i < len(layers) - 1:
            H = np.tanh(Z)
            cache.append(H)
        else:
            H = Z
    return H, cache


def backward(W, cache, dY):
    """Gradient of a scalar loss with respect to the packed parameters, given
    dL/dY; returns the packed gradient."""
    layers = unpack(W)
    grads = [None] * len(layers)
    G = np.asarray(dY, dtype=np.float64)
    for i in range(len(layers) - 1, -1, -1):
        Wl, _ = layers[i]
        Hin = cache[i]
        grads[i] = (Hin.T @ G, G.sum(axis=0))
        if i > 0:
            G = (G @ Wl.T) * (1.0 - cache[i] ** 2)
    return pack(grads)


def mse_loss(Y, T):
    """L = mean((Y - T)^2) over batch and outputs, and dL/dY."""
    D = Y - T
    return float(np.mean(D * D)), 2.0 * D / D.size


def adam_step(W, dW, m1, m2, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update; returns new (W, m1, m2)."""
    m1 = beta1 * m1 + (1.0 - beta1) * dW
    m2 = beta2 * m2 + (1.0 - beta2) * dW * dW
    mhat = m1 / (1.0 - beta1 ** t)
    vhat = m2 / (1.0 - beta2 ** t)
    return W - lr * mhat / (np.sqrt(vhat) + eps), m1, m2
