"""Pins of the oracle's accelerations (O8: g = -grad phi, term by term).

* the direct acceleration equals central finite differences of the direct
  potential evaluated at displaced points (a separate routine);
* momentum conservation: sum_i m_i g_i = 0 for the direct sum;
* outside a uniform sphere with no ambient medium, g -> -G M r / |r|^3;
* theta -> 0 opens every node: the tree acceleration equals the direct one;
* convergence orders of a single far node: the monopole's relative error
  falls as (l/d)^2, monopole + quadrupole as (l/d)^3 (a dropped or mis-signed
  quadrupole-gradient term breaks the second slope).
"""
import math

import numpy as np
import pytest

from amr_inputs import random_amr, uniform_sphere
from oracle import OracleTree

from test_oracle_bh import _corner_mass_grid


def _positions(t):
    x, y, z, m = t.cells()
    return np.stack([x, y, z], 1), m


def test_direct_accel_is_minus_gradient_of_direct_potential():
    g = random_amr(41, nbase=2, max_level=2, p_refine=0.3, zero_fraction=0.1)
    t = OracleTree(g)
    P, m = _positions(t)
    rng = np.random.default_rng(2)
    tg = rng.choice(t.ncells, 20, replace=False)
    acc = t.direct_accel(tg)
    hmin = g.box_size / (8 * 2 * (1 << 2))
    step = 1e-4 * hmin
    for k in range(3):
        e = np.zeros(3)
        e[k] = step
        fd = -(t.direct_at(P[tg] + e, tg) - t.direct_at(P[tg] - e, tg)) / (2 * step)
        scale = np.linalg.norm(acc, axis=1)
        assert np.all(np.abs(acc[:, k] - fd) <= 1e-6 * scale), np.max(np.abs(acc[:, k] - fd) / scale)


def test_direct_accel_conserves_momentum():
    g = random_amr(42, nbase=1, max_level=2, p_refine=0.5, zero_fraction=0.1)
    t = OracleTree(g)
    _, m = _positions(t)
    acc = t.direct_accel()
    total = (m[:, None] * acc).sum(0)
    assert np.all(np.abs(total) <= 1e-12 * (m[:, None] * np.abs(acc)).sum(0))


def test_uniform_sphere_exterior_field():
    g = uniform_sphere(radius=0.3, rho_in=1.0, rho_out=0.0)
    t = OracleTree(g)
    P, m = _positions(t)
    r = P - 0.5
    rn = np.linalg.norm(r, axis=1)
    sel = np.nonzero(rn > 0.42)[0]
    sel = sel[np.random.default_rng(0).choice(sel.size, 200, replace=False)]
    acc = t.direct_accel(sel)
    want = -m.sum() * r[sel] / rn[sel, None] ** 3
    err = np.linalg.norm(acc - want, axis=1) / np.linalg.norm(want, axis=1)
    assert err.max() <= 5e-3, err.max()
    # pointing inward
    assert np.all(np.einsum("ij,ij->i", acc, r[sel]) < 0)


def test_theta_to_zero_accel_is_direct():
    g = random_amr(43, nbase=2, max_level=2, p_refine=0.3, zero_fraction=0.1)
    t = OracleTree(g)
    t.walk(64, 1e-6)
    acc = t.accel().reshape(-1, 3)
    rng = np.random.default_rng(5)
    tg = rng.choice(t.ncells, 40, replace=False)
    ref = t.direct_accel(tg)
    scale = np.linalg.norm(ref, axis=1)
    assert np.max(np.linalg.norm(acc[tg] - ref, axis=1) / scale) <= 1e-12


def test_group_subset_accel_equals_full_accel():
    g = random_amr(44, nbase=2, max_level=2, p_refine=0.3, zero_fraction=0.1)
    t = OracleTree(g)
    t.walk(64, 0.6)
    full = t.accel().reshape(-1, 3)
    groups = np.array([0, 5, t.n_groups(64) - 1])
    sub, counts = t.solve_groups_accel(groups, theta=0.6)
    m = np.arange(64)
    for q, gi in enumerate(groups):
        leaf, s = divmod(int(gi), 8)
        mm = s * 64 + m
        i = sum(((mm >> (3 * p)) & 1) << p for p in range(3))
        j = sum(((mm >> (3 * p + 1)) & 1) << p for p in range(3))
        k = sum(((mm >> (3 * p + 2)) & 1) << p for p in range(3))
        assert np.array_equal(sub[q], full[leaf * 512 + k * 64 + j * 8 + i])


@pytest.mark.parametrize("order,slope", [(0, 2.0), (2, 3.0)])
def test_far_node_accel_convergence_order(order, slope):
    g = _corner_mass_grid()
    t = OracleTree(g)
    t.walk(1, 1.0)
    acc = t.accel(order=order).reshape(-1, 3)
    P, m = _positions(t)
    exact = t.direct_accel()
    l = 1.0 / 32
    mo = t.moments()
    root = int(np.nonzero(mo["key"] == np.uint64(0))[0][0])
    d = np.linalg.norm(P - mo["X"][root], axis=1)
    rel = np.linalg.norm(acc - exact, axis=1) / np.linalg.norm(exact, axis=1)
    ds, es = [], []
    for lo_ in np.geomspace(4 * l, 24 * l, 8):
        sel = (d > lo_) & (d < lo_ * 1.15)
        if sel.sum() >= 5:
            ds.append(np.median(d[sel]))
            es.append(np.median(rel[sel]))
    fit = np.polyfit(np.log(ds), np.log(es), 1)[0]
    assert abs(-fit - slope) <= 0.25, (fit, ds, es)
