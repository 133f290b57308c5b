"""Pins of the FP64 network and feature oracles used by the learned-theta tests.

* analytic gradient = central finite differences of the loss (FP64);
* Adam's first step is -lr g / (|g| + eps) (closed form, since m^ = g, v^ = g^2);
* the output stays in (0.2, 1.0); bf16 rounding on known values;
* features of a uniform-density grid take their closed-form values.
"""
import numpy as np
import pytest

from amr_inputs import random_amr, uniform_sphere
from amr_inputs.mlp_init import N_PARAMS, glorot_init
from oracle import OracleTree
from oracle import mlp
from oracle.features import group_features


def _data(n=37, seed=0):
    rng = np.random.default_rng(seed)
    X = rng.normal(size=(n, 12)) * 3 + 1
    y = rng.uniform(0.2, 1.0, n)
    mean = rng.normal(size=12)
    scale = rng.uniform(0.2, 2.0, 12)
    return X, y, mean, scale


def test_gradient_matches_finite_differences():
    p = glorot_init(3) + np.random.default_rng(1).normal(scale=0.05, size=N_PARAMS)
    X, y, mean, scale = _data()
    g = mlp.grad(p, X, y, mean, scale)
    h = 1e-6
    rng = np.random.default_rng(2)
    idx = np.concatenate([rng.choice(N_PARAMS, 300, replace=False), [N_PARAMS - 1, 0, 768, 832, 4928, 4992]])
    for i in idx:
        e = np.zeros(N_PARAMS)
        e[i] = h
        fd = (mlp.loss(p + e, X, y, mean, scale) - mlp.loss(p - e, X, y, mean, scale)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-7 * max(1.0, np.abs(g).max()), (i, fd, g[i])


def test_adam_first_step_closed_form():
    rng = np.random.default_rng(4)
    p = rng.normal(size=50)
    g = rng.normal(size=50)
    p1, m, v = mlp.adam_step(p, g, np.zeros(50), np.zeros(50), 1, lr=1e-2)
    assert np.allclose(p1 - p, -1e-2 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=0)
    # a second step with the same gradient moves by the same amount again
    p2, _, _ = mlp.adam_step(p1, g, m, v, 2, lr=1e-2)
    assert np.allclose(p2 - p1, -1e-2 * g / (np.abs(g) + 1e-8), rtol=1e-10, atol=0)


def test_output_range_and_bf16_rounding():
    X, y, mean, scale = _data(200)
    th, _ = mlp.forward(glorot_init(7) * 20, X * 50, mean, scale)  # saturated
    assert np.all(th >= 0.2) and np.all(th <= 1.0) and th.min() == 0.2 and th.max() == 1.0
    th, _ = mlp.forward(glorot_init(7), X, mean, scale)
    assert np.all(th > 0.2) and np.all(th < 1.0)
    vals = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -9, -2.5, 3.0e-3], np.float32)
    r = mlp.bf16_round(vals)
    assert r[0] == 1.0 and r[1] == 1.0 and r[2] == 1.0 + 2 ** -7 and r[3] == -2.5
    assert abs(r[4] - 3.0e-3) <= 3.0e-3 * 2 ** -8


def test_features_of_a_uniform_grid():
    g = uniform_sphere(nbase=2, rho_in=1.0, rho_out=1.0)  # uniform density
    t = OracleTree(g)
    F = group_features(t, g)
    assert F.shape == (g.nleaf * 8, 12)
    assert np.all(F[:, 0] == 6.0)
    assert np.allclose(F[:, 1], np.log(64 / 4096.0), atol=1e-12)  # every group holds 64 of 4096 equal masses
    assert np.allclose(F[:, 2], np.log(4 / 16.0), atol=1e-12)
    assert np.all(F[:, 3] == 0)
    assert np.allclose(F[:, 4], 0.0, atol=1e-12)
    assert np.allclose(F[:, 5:11], np.log(1e-6), atol=1e-6)
    assert np.allclose(F[:, 11], 0.0, atol=1e-12)


def test_features_are_finite_with_empty_blocks():
    g = random_amr(21, nbase=2, max_level=3, zero_fraction=0.2)
    F = group_features(OracleTree(g), g)
    assert np.isfinite(F).all()
    assert F[:, 3].max() == 3


def test_bf16_forward_and_snap():
    X, y, mean, scale = _data(300)
    p = glorot_init(9)
    th, _ = mlp.forward(p, X, mean, scale)
    tb = mlp.forward_bf16(p, X, mean, scale)
    # bf16 inputs, weights and activations move theta by well under the grid step
    assert np.max(np.abs(tb - th)) <= 0.01 and np.max(np.abs(tb - th)) > 0
    # weights and inputs that bf16 holds exactly, hidden layers saturated (tanh = +-1 exactly in bf16):
    # the bf16 forward is the fp64 forward
    W1, b1, W2, b2, W3, b3 = mlp.unpack(glorot_init(5))
    W1 = np.where(W1 < 0, -4.0, 4.0)
    W2 = np.where(W2 < 0, -32.0, 32.0)
    W3 = np.round(W3 * 64) / 64
    q = mlp.pack(W1, np.zeros(64), W2, np.zeros(64), W3, 0.25)
    Xe = np.where(X < 0, -4.0, 4.0)  # pre-activations are multiples of 32: tanh is 0 or +-1 exactly
    assert np.array_equal(mlp.forward_bf16(q, Xe, np.zeros(12), np.ones(12)),
                          mlp.forward(q, Xe, np.zeros(12), np.ones(12))[0])
    s = mlp.snap_up(np.array([0.2, 0.2 + 5e-7, 0.21, 0.25, 0.2500001, 0.26, 0.999, 1.0, 0.1, 0.55]))
    assert np.allclose(s, [0.2, 0.2, 0.25, 0.25, 0.25, 0.3, 1.0, 1.0, 0.2, 0.55], atol=1e-12, rtol=0)
    assert np.allclose(mlp.snap_up(np.array([0.61, 0.7]), shift=0.1), [0.55, 0.6], atol=1e-12, rtol=0)
