"""The branching scorer's multilayer perceptron in float64 (test oracle).

Architecture: x (32) -> h1 = relu(W1 x + b1) (128) -> h2 = relu(W2 h1 + b2)
(128) -> y = w3 . h2 + b3.  Loss: mean squared error over rows.  Optimizer:
Adam (Kingma & Ba): m <- b1 m + (1-b1) g; v <- b2 v + (1-b2) g^2;
p <- p - lr * (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).

Weights and inputs arrive as bfloat16 bit patterns; decoding them is exact
(a bfloat16 is the upper 16 bits of a float32), so the oracle evaluates the
very numbers the device holds, in float64.
"""
from __future__ import annotations

import numpy as np

N_IN, N_H = 32, 128


def decode_bf16(bits):
    bits = np.asarray(bits, dtype=np.uint16)
    return (bits.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def forward(X, W1, b1, W2, b2, w3, b3):
    """Returns (y, h1, h2) for rows X [R, 32]."""
    h1 = np.maximum(X @ W1.T + b1, 0.0)
    h2 = np.maximum(h1 @ W2.T + b2, 0.0)
    y = h2 @ w3 + b3
    return y, h1, h2


def loss_and_grads(X, t, W1, b1, W2, b2, w3, b3):
    """MSE loss and its gradient with respect to every parameter."""
    R = X.shape[0]
    z1 = X @ W1.T + b1
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ W2.T + b2
    h2 = np.maximum(z2, 0.0)
    y = h2 @ w3 + b3
    loss = float(np.mean((y - t) ** 2))
    dy = 2.0 * (y - t) / R
    dw3 = h2.T @ dy
    db3 = float(dy.sum())
    dz2 = np.outer(dy, w3) * (z2 > 0)
    dW2 = dz2.T @ h1
    db2 = dz2.sum(axis=0)
    dz1 = (dz2 @ W2) * (z1 > 0)
    dW1 = dz1.T @ X
    db1 = dz1.sum(axis=0)
    return loss, dict(W1=dW1, b1=db1, W2=dW2, b2=db2, w3=dw3, b3=db3)


def adam_step(p, g, m, v, lr, t, beta1=0.9, beta2=0.999, eps=1e-8):
    m = beta1 * m + (1 - beta1) * g
    v = beta2 * v + (1 - beta2) * g * g
    mhat = m / (1 - beta1 ** t)
    vhat = v / (1 - beta2 ** t)
    return p - lr * mhat / (np.sqrt(vhat) + eps), m, v


def encode_bf16(x):
    """float -> bfloat16 bit pattern by the definition of round to nearest,
    ties to even: keep the upper 16 bits of the float32, adding one unit in
    the last kept place when the dropped half-word exceeds one half, or equals
    one half and the kept part is odd."""
    u = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.int64)
    hi, lo = u >> 16, u & 0xFFFF
    up = (lo > 0x8000) | ((lo == 0x8000) & (hi & 1 == 1))
    return (hi + up).astype(np.uint16)
