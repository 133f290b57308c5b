"""Pins of the oracle's direct sum (O2: Eq. 2 of section 1, read without the 1/2).

Each check is independent of the oracle's own arithmetic: exact two-body
values, 40-digit mpmath brute force, grid symmetries, reciprocity computed with
a numpy pair matrix, and translation invariance.
"""
import mpmath
import numpy as np
import pytest

from amr_inputs import build_grid, random_amr, single_block, uniform_sphere
from oracle import OracleTree


def _two_cell_grid():
    def dens(lo, h):
        r = np.zeros((lo.shape[0], 8, 8, 8))
        r[0, 1, 2, 3] = 3.0     # cell x=3, y=2, z=1
        r[0, 6, 5, 0] = 0.5     # cell x=0, y=5, z=6
        return r
    return build_grid("two_cells", 1, lambda *a: False, 0, dens)


def test_two_cells_exact():
    g = _two_cell_grid()
    t = OracleTree(g)
    h = 1.0 / 8
    m1, m2 = 3.0 * h ** 3, 0.5 * h ** 3
    r1 = np.array([3.5, 2.5, 1.5]) * h
    r2 = np.array([0.5, 5.5, 6.5]) * h
    d = np.linalg.norm(r1 - r2)
    c1 = 1 * 64 + 2 * 8 + 3
    c2 = 6 * 64 + 5 * 8 + 0
    phi = t.direct([c1, c2], G=2.0)
    assert phi[0] == pytest.approx(-2.0 * m2 / d, rel=1e-15)
    assert phi[1] == pytest.approx(-2.0 * m1 / d, rel=1e-15)
    # any other cell sees both masses
    phi3 = t.direct([0], G=1.0)[0]
    r0 = np.array([0.5, 0.5, 0.5]) * h
    assert phi3 == pytest.approx(-(m1 / np.linalg.norm(r0 - r1) + m2 / np.linalg.norm(r0 - r2)), rel=1e-15)


def _mp_direct(x, y, z, m, targets, G=1.0):
    mpmath.mp.dps = 40
    X = [mpmath.mpf(float(v)) for v in x]
    Y = [mpmath.mpf(float(v)) for v in y]
    Z = [mpmath.mpf(float(v)) for v in z]
    Mm = [mpmath.mpf(float(v)) for v in m]
    out = []
    for i in targets:
        s = mpmath.mpf(0)
        for j in range(len(X)):
            if j == i or Mm[j] == 0:
                continue
            s += Mm[j] / mpmath.sqrt((X[i] - X[j]) ** 2 + (Y[i] - Y[j]) ** 2 + (Z[i] - Z[j]) ** 2)
        out.append(float(-G * s))
    return np.array(out)


def test_direct_vs_mpmath_single_block():
    g = single_block(seed=4, sigma=1.0)
    t = OracleTree(g)
    x, y, z, m = t.cells()
    # cell geometry is the definition O1: lo + (i + 1/2) h, m = rho h^3
    cc = g.cell_centres().reshape(-1, 3)
    assert np.array_equal(x, cc[:, 0]) and np.array_equal(y, cc[:, 1]) and np.array_equal(z, cc[:, 2])
    assert np.allclose(m, g.rho.ravel() * (1.0 / 8) ** 3, rtol=1e-15, atol=0)
    targets = [0, 7, 63, 100, 255, 256, 400, 511]
    ref = _mp_direct(x, y, z, m, targets)
    got = t.direct(targets)
    assert np.max(np.abs(got - ref) / np.abs(ref)) <= 1e-14


def test_direct_vs_mpmath_amr():
    g = random_amr(11, nbase=2, max_level=1, p_refine=0.25)
    t = OracleTree(g)
    x, y, z, m = t.cells()
    rng = np.random.default_rng(0)
    targets = sorted(rng.choice(t.ncells, 6, replace=False).tolist())
    ref = _mp_direct(x, y, z, m, targets)
    got = t.direct(targets)
    assert np.max(np.abs(got - ref) / np.abs(ref)) <= 1e-14


def test_direct_symmetry_reciprocity_translation():
    g = uniform_sphere(nbase=2)  # 16^3 cells, symmetric under the cube group about the centre
    t = OracleTree(g)
    phi = t.direct().reshape(8, 8, 8, 8)
    # assemble the 16^3 field from the 2x2x2 blocks
    field = np.zeros((16, 16, 16))
    leaves = g.leaf_blocks
    for f, b in enumerate(leaves):
        i0, j0, k0 = (np.round(g.lo[b] * 16)).astype(int)
        field[k0:k0 + 8, j0:j0 + 8, i0:i0 + 8] = phi[f]
    scale = np.abs(field).max()
    for sym in (field.transpose(0, 2, 1), field.transpose(1, 0, 2), field.transpose(2, 1, 0),
                field[::-1], field[:, ::-1], field[:, :, ::-1]):
        assert np.max(np.abs(sym - field)) <= 1e-14 * scale
    # reciprocity: sum_i m_i phi_i = -G sum_{i != j} m_i m_j / r_ij (numpy pair matrix)
    x, y, z, m = t.cells()
    P = np.stack([x, y, z], 1)
    D = np.sqrt(((P[:, None, :] - P[None, :, :]) ** 2).sum(-1))
    np.fill_diagonal(D, np.inf)
    W_pairs = -np.sum(m[:, None] * m[None, :] / D)
    W = np.sum(m * t.direct())
    assert W == pytest.approx(W_pairs, rel=1e-13)
    # translation invariance: shift the box by a dyadic offset
    g2 = uniform_sphere(nbase=2)
    g2.box_lo = g2.box_lo + np.array([0.25, -0.5, 1.0])
    g2.lo = g2.lo + np.array([0.25, -0.5, 1.0])
    t2 = OracleTree(g2)
    assert np.max(np.abs(t2.direct() - t.direct())) <= 1e-14 * scale
