"""Closed-form pins of the oracle's per-group features 1-11 (oracle/features.py).

The features read node moments (the centre of mass of the centres-of-gravitation
kernel, section 3.2.3, and the offset delta and edge l of Eq. THETA2, section 2)
of three nodes per group: the group's own 4^3 node, its leaf block and the leaf
block's parent.  A uniform grid makes most of them constant, so these pins use
hand-placed point masses whose moments are known exactly:

* one cell: centre of mass at the cell centre, Q = 0, delta = |r - c|;
* two cells of masses m1, m2 at separation d: Q = (m1 m2 / M)(3 d d^T - |d|^2 I),
  whose Frobenius norm is (m1 m2 / M) sqrt(6) |d|^2 (eigenvalues 2, -1, -1 times
  |d|^2), so ||Q||_F / (M l^2) = (m1 m2 / M^2) sqrt(6) |d|^2 / l^2;
* a density linear in x inside one block: the moments separate per axis and
  are sums over 4 or 8 values.

Each pin fails for a plausible slip in the feature code: the wrong ancestor
node, M l instead of M l^2, the off-diagonal weights of the Frobenius norm, the
max/mean or the density-contrast ratio.
"""
import math

import numpy as np

from amr_inputs.grids import build_grid
from oracle import OracleTree
from oracle.features import group_features

EPS = 1e-6
LOG_TINY = math.log(1e-30)


def _grid():
    """nbase 2, the level-0 block at the origin refined once: 7 level-0 leaves, then 8 level-1 leaves."""
    def refine(L, lo, e):
        return L == 0 and np.allclose(lo, 0.0)

    g = build_grid("feature_pins", 2, refine, 1, lambda lo, h: np.zeros((lo.shape[0], 8, 8, 8)))
    return g


def _leaf(g, level, lo):
    lb = g.leaf_blocks
    for n, b in enumerate(lb):
        if g.level[b] == level and np.allclose(g.lo[b], lo):
            return n
    raise KeyError((level, lo))


def _geom(g, leaf):
    b = g.leaf_blocks[leaf]
    edge = g.box_size / (g.nbase * 2.0 ** g.level[b])
    return g.lo[b].copy(), edge, edge / 8


def _cell_centre(g, leaf, i, j, k):
    lo, _, h = _geom(g, leaf)
    return lo + (np.array([i, j, k]) + 0.5) * h


def _sub(i, j, k):
    return (i >> 2) | ((j >> 2) << 1) | ((k >> 2) << 2)


def _group_centre(g, leaf, sub):
    lo, _, h = _geom(g, leaf)
    return lo + (4 * np.array([sub & 1, (sub >> 1) & 1, (sub >> 2) & 1]) + 2) * h


def _put(g, leaf, i, j, k, mass):
    _, _, h = _geom(g, leaf)
    g.rho[leaf, k, j, i] = mass / h ** 3


def _feat(g):
    return group_features(OracleTree(g), g)


def test_one_point_mass():
    g = _grid()
    leaf = _leaf(g, 1, (0.25, 0.25, 0.25))  # octant 7 of the refined block
    i, j, k = 1, 6, 3
    _put(g, leaf, i, j, k, 2.5)
    F = _feat(g)
    r = _cell_centre(g, leaf, i, j, k)
    lo, lb_edge, h = _geom(g, leaf)
    sub = _sub(i, j, k)
    row = leaf * 8 + sub
    cg, cb, cp = _group_centre(g, leaf, sub), lo + lb_edge / 2, np.full(3, 0.25)
    want = {
        0: 6.0, 1: 0.0, 2: math.log(4 * h), 3: 1.0, 4: math.log(64.0),
        5: math.log(np.linalg.norm(r - cg) / (4 * h) + EPS), 6: math.log(EPS),
        7: math.log(np.linalg.norm(r - cb) / lb_edge + EPS), 8: math.log(EPS),
        9: math.log(np.linalg.norm(r - cp) / 0.5 + EPS), 10: math.log(EPS),
        11: math.log(8.0),
    }
    for c, v in want.items():
        assert abs(F[row, c] - v) <= 1e-12, (c, F[row, c], v)
    # the other groups of the block: no mass of their own, same block and parent
    for s in range(8):
        if s == sub:
            continue
        q = leaf * 8 + s
        assert F[q, 1] == LOG_TINY and F[q, 4] == 0.0 and F[q, 11] == LOG_TINY
        assert abs(F[q, 5] - math.log(EPS)) <= 1e-12 and abs(F[q, 6] - math.log(EPS)) <= 1e-12
        assert np.allclose(F[q, 7:11], F[row, 7:11], rtol=0, atol=1e-12)
    # a sibling level-1 leaf: massless block, same parent node
    sib = _leaf(g, 1, (0.0, 0.0, 0.0))
    assert abs(F[sib * 8, 7] - math.log(EPS)) <= 1e-12
    assert abs(F[sib * 8, 9] - want[9]) <= 1e-12
    # a level-0 leaf: its parent is the root (edge 1, centre 0.5)
    base = _leaf(g, 0, (0.5, 0.5, 0.5))
    assert F[base * 8, 3] == 0.0 and abs(F[base * 8, 2] - math.log(4 / 16.0)) <= 1e-12
    assert abs(F[base * 8, 9] - math.log(np.linalg.norm(r - 0.5) / 1.0 + EPS)) <= 1e-12
    assert abs(F[base * 8, 10] - math.log(EPS)) <= 1e-12


def _two_mass_q(m1, m2, d, l):
    M = m1 + m2
    return m1 * m2 / M ** 2 * math.sqrt(6.0) * float(d @ d) / l ** 2


def test_two_masses_in_one_group():
    g = _grid()
    leaf = _leaf(g, 0, (0.5, 0.0, 0.5))
    (i1, j1, k1), (i2, j2, k2) = (0, 0, 0), (3, 2, 1)  # separation not along an axis: Q has off-diagonals
    m1, m2 = 1.0, 3.0
    _put(g, leaf, i1, j1, k1, m1)
    _put(g, leaf, i2, j2, k2, m2)
    F = _feat(g)
    r1, r2 = _cell_centre(g, leaf, i1, j1, k1), _cell_centre(g, leaf, i2, j2, k2)
    X = (m1 * r1 + m2 * r2) / (m1 + m2)
    d = r2 - r1
    lo, lb_edge, h = _geom(g, leaf)
    row = leaf * 8 + 0
    cg, cb = _group_centre(g, leaf, 0), lo + lb_edge / 2
    want = {
        1: 0.0, 4: math.log(m2 / ((m1 + m2) / 64)),
        5: math.log(np.linalg.norm(X - cg) / (4 * h) + EPS),
        6: math.log(_two_mass_q(m1, m2, d, 4 * h) + EPS),
        7: math.log(np.linalg.norm(X - cb) / lb_edge + EPS),
        8: math.log(_two_mass_q(m1, m2, d, lb_edge) + EPS),
        9: math.log(np.linalg.norm(X - 0.5) + EPS),
        10: math.log(_two_mass_q(m1, m2, d, 1.0) + EPS),
        11: math.log(8.0),
    }
    for c, v in want.items():
        assert abs(F[row, c] - v) <= 1e-12, (c, F[row, c], v)
    # an axis-aligned pair gives a different (diagonal) Q with the same formula
    g2 = _grid()
    _put(g2, leaf, 0, 0, 0, m1)
    _put(g2, leaf, 3, 0, 0, m2)
    F2 = _feat(g2)
    d2 = np.array([3 * h, 0.0, 0.0])
    assert abs(F2[row, 6] - math.log(_two_mass_q(m1, m2, d2, 4 * h) + EPS)) <= 1e-12


def test_masses_in_two_blocks_under_one_parent():
    g = _grid()
    a = _leaf(g, 1, (0.0, 0.25, 0.0))
    b = _leaf(g, 1, (0.25, 0.0, 0.25))
    m1, m2 = 2.0, 0.5
    _put(g, a, 5, 1, 2, m1)
    _put(g, b, 2, 7, 6, m2)
    F = _feat(g)
    r1, r2 = _cell_centre(g, a, 5, 1, 2), _cell_centre(g, b, 2, 7, 6)
    X = (m1 * r1 + m2 * r2) / (m1 + m2)
    for leaf, r, (i, j, k), m in ((a, r1, (5, 1, 2), m1), (b, r2, (2, 7, 6), m2)):
        lo, lb_edge, h = _geom(g, leaf)
        row = leaf * 8 + _sub(i, j, k)
        # group and block hold one mass each: a point mass
        assert abs(F[row, 1] - math.log(m / (m1 + m2))) <= 1e-12
        assert abs(F[row, 7] - math.log(np.linalg.norm(r - (lo + lb_edge / 2)) / lb_edge + EPS)) <= 1e-12
        assert abs(F[row, 8] - math.log(EPS)) <= 1e-12
        # the parent (the refined level-0 block, edge 0.5, centre 0.25) holds both
        assert abs(F[row, 9] - math.log(np.linalg.norm(X - 0.25) / 0.5 + EPS)) <= 1e-12
        assert abs(F[row, 10] - math.log(_two_mass_q(m1, m2, r2 - r1, 0.5) + EPS)) <= 1e-12
        assert abs(F[row, 11] - math.log(8.0)) <= 1e-12


def test_density_linear_in_x():
    g = _grid()
    leaf = _leaf(g, 0, (0.5, 0.5, 0.0))
    lo, lb_edge, h = _geom(g, leaf)
    w8 = 1.0 + np.arange(8)  # density 1 + i in cell column i
    g.rho[leaf] = w8[None, None, :]
    F = _feat(g)
    offs = (np.arange(4) + 0.5) * h  # cell offsets inside a group, per axis
    syy = 4 * float(((offs - 2 * h) ** 2).sum())  # sum over a 4x4 (j, k) face of (y - Y)^2 per unit x-weight
    for sub in range(8):
        ix = sub & 1
        w = w8[4 * ix:4 * ix + 4]
        row = leaf * 8 + sub
        # max / mean over the 64 cells (uniform in y, z)
        assert abs(F[row, 4] - math.log(w.max() / w.mean())) <= 1e-12
        # density contrast against the block's mean
        assert abs(F[row, 11] - math.log(w.mean() / w8.mean())) <= 1e-12
        # centre of mass offset: along x only
        X = float((w * offs).sum() / w.sum())
        assert abs(F[row, 5] - math.log(abs(X - 2 * h) / (4 * h) + EPS)) <= 1e-12
        # quadrupole: diagonal, from per-axis second moments (mass per cell = rho h^3)
        sxx = 16 * float((w * (offs - X) ** 2).sum()) * h ** 3
        s_yz = float(w.sum()) * syy * h ** 3
        q = np.array([2 * sxx - 2 * s_yz, 2 * s_yz - sxx - s_yz, 2 * s_yz - sxx - s_yz])
        M = 16 * float(w.sum()) * h ** 3
        want = math.log(float(np.sqrt((q ** 2).sum())) / (M * (4 * h) ** 2) + EPS)
        assert abs(F[row, 6] - want) <= 1e-11, (sub, F[row, 6], want)
