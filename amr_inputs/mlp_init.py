"""Seeded initial parameters for the 12 -> 64 -> 64 -> 1 opening-angle network.

Random numbers only (Glorot-uniform weights, zero biases); the network's
arithmetic lives elsewhere.  Layout: W1[64][12] | b1[64] | W2[64][64] | b2[64]
| W3[64] | b3.
"""
import numpy as np

N_IN, N_H = 12, 64
N_PARAMS = N_H * N_IN + N_H + N_H * N_H + N_H + N_H + 1


def glorot_init(seed: int = 42) -> np.ndarray:
    rng = np.random.default_rng(seed)

    def glorot(fan_out, fan_in):
        a = np.sqrt(6.0 / (fan_in + fan_out))
        return rng.uniform(-a, a, size=(fan_out, fan_in))

    parts = [glorot(N_H, N_IN).ravel(), np.zeros(N_H), glorot(N_H, N_H).ravel(), np.zeros(N_H),
             glorot(1, N_H).ravel(), np.zeros(1)]
    p = np.concatenate(parts)
    assert p.size == N_PARAMS
    return p
