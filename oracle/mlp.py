"""FP64 oracle of the per-group opening-angle network (test infrastructure only).

The network of the learned-theta part (an addition to the paper's single
runtime theta): x' = (x - mean) * scale; h1 = tanh(W1 x' + b1);
h2 = tanh(W2 h1 + b2); z = W3 . h2 + b3; theta = 0.2 + 0.8 sigmoid(z);
loss L = mean_s (theta_s - y_s)^2; Adam (Kingma & Ba 2015).  Parameter layout:
W1[64][12] | b1[64] | W2[64][64] | b2[64] | W3[64] | b3.
Pinned by central finite differences and by Adam's closed-form first step.
"""
from __future__ import annotations

import numpy as np

N_IN, N_H = 12, 64
N_PARAMS = N_H * N_IN + N_H + N_H * N_H + N_H + N_H + 1


def unpack(p):
    p = np.asarray(p, np.float64)
    o = 0
    W1 = p[o:o + N_H * N_IN].reshape(N_H, N_IN); o += N_H * N_IN
    b1 = p[o:o + N_H]; o += N_H
    W2 = p[o:o + N_H * N_H].reshape(N_H, N_H); o += N_H * N_H
    b2 = p[o:o + N_H]; o += N_H
    W3 = p[o:o + N_H]; o += N_H
    b3 = p[o]
    return W1, b1, W2, b2, W3, b3


def pack(W1, b1, W2, b2, W3, b3):
    return np.concatenate([W1.ravel(), b1, W2.ravel(), b2, W3, np.atleast_1d(b3)])


def forward(p, X, mean, scale):
    W1, b1, W2, b2, W3, b3 = unpack(p)
    Xn = (np.asarray(X, np.float64) - mean) * scale
    H1 = np.tanh(Xn @ W1.T + b1)
    H2 = np.tanh(H1 @ W2.T + b2)
    z = H2 @ W3 + b3
    s = 1.0 / (1.0 + np.exp(-z))
    return 0.2 + 0.8 * s, dict(Xn=Xn, H1=H1, H2=H2, s=s)


def loss(p, X, y, mean, scale):
    th, _ = forward(p, X, mean, scale)
    return float(np.mean((th - y) ** 2))


def grad(p, X, y, mean, scale):
    """Analytic gradient of loss() by the chain rule."""
    W1, b1, W2, b2, W3, b3 = unpack(p)
    th, c = forward(p, X, mean, scale)
    n = len(y)
    dth = 2.0 * (th - y) / n
    dz = dth * 0.8 * c["s"] * (1.0 - c["s"])
    gW3 = c["H2"].T @ dz
    gb3 = dz.sum()
    d2 = np.outer(dz, W3) * (1.0 - c["H2"] ** 2)
    gW2 = d2.T @ c["H1"]
    gb2 = d2.sum(0)
    d1 = (d2 @ W2) * (1.0 - c["H1"] ** 2)
    gW1 = d1.T @ c["Xn"]
    gb1 = d1.sum(0)
    return pack(gW1, gb1, gW2, gb2, gW3, gb3)


def adam_step(p, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """Returns new (p, m, v) after Adam step number t (t >= 1)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


def bf16_round(x):
    """Round float32 values to bfloat16 (nearest even), returned as float64."""
    u = np.asarray(x, np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def forward_bf16(p, X, mean, scale):
    """The network as its bf16 inference evaluates it: standardised inputs,
    weights, biases and both hidden activations rounded to bfloat16, every
    product and sum in fp64 (the kernels accumulate in fp32).  Returns theta."""
    W1, b1, W2, b2, W3, b3 = (bf16_round(np.asarray(a, np.float32)) for a in unpack(p))
    Xn = bf16_round(((np.asarray(X, np.float64) - mean) * scale).astype(np.float32))
    H1 = bf16_round(np.tanh(Xn @ W1.T + b1).astype(np.float32))
    H2 = bf16_round(np.tanh(H1 @ W2.T + b2).astype(np.float32))
    z = H2 @ W3 + b3
    s = 1.0 / (1.0 + np.exp(-z))
    return 0.2 + 0.8 * s


def snap_up(theta, shift=0.0):
    """theta - shift moved up to the next value of the grid 0.20, 0.25, ..., 1.00
    (values within 1e-6 above a grid value stay on it; the grid's ends clamp)."""
    k = np.clip(np.ceil((np.asarray(theta, np.float64) - shift - 1e-6 - 0.2) * 20.0), 0, 16)
    return 0.2 + 0.05 * k
