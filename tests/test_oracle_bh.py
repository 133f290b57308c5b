"""Pins of the oracle's Barnes-Hut result (O4-O7).

* theta -> 0 opens everything: exactly the direct sum (the paper's error
  figure uses alpha = 0 for the direct algorithm);
* group size 1 equals a textbook per-particle Barnes-Hut written here
  independently (classic top-down octree of the cell centres, recursive walk);
* convergence orders of a single far node: monopole (l/d)^2, monopole +
  quadrupole (l/d)^3;
* list invariants: every massive cell covered exactly once per group, no
  accepted node containing a group cell;
* error grows with theta and is at the percent level at theta = 1 (section 2).
"""
import math

import numpy as np
import pytest

from amr_inputs import build_grid, maclaurin_spheroid, random_amr, single_block, uniform_sphere
from oracle import OracleTree
from oracle.oracle import split_key


def test_theta_to_zero_is_direct():
    g = random_amr(21, nbase=2, max_level=2, p_refine=0.3, zero_fraction=0.1)
    t = OracleTree(g)
    w = t.walk(64, 1e-6)
    assert w["n_far"].sum() == 0
    phi = t.potential().ravel()
    d = t.direct()
    assert np.max(np.abs(phi - d) / np.abs(d)) <= 1e-13


def _textbook_bh(P, m, box_lo, box, theta, targets):
    """Classic per-particle Barnes-Hut on the cell centres (independent code)."""
    cache = {}

    def moments(lo, e):
        key = (round(lo[0] / e * 2), round(lo[1] / e * 2), round(lo[2] / e * 2), e)
        if key not in cache:
            sel = np.all((P >= lo) & (P < lo + e), axis=1)
            idx = np.nonzero(sel)[0]
            M = m[idx].sum()
            if M > 0:
                X = (m[idx, None] * P[idx]).sum(0) / M
                D = P[idx] - X
                Q = 3 * np.einsum("i,ij,ik->jk", m[idx], D, D) - np.eye(3) * np.sum(m[idx] * (D * D).sum(1))
            else:
                X, Q = lo + 0.5 * e, np.zeros((3, 3))
            cache[key] = (idx, M, X, Q)
        return cache[key]

    out = []
    for i in targets:
        acc = 0.0
        stack = [(np.asarray(box_lo, float), float(box))]
        while stack:
            lo, e = stack.pop()
            idx, M, X, Q = moments(lo, e)
            if M == 0:
                continue
            if len(idx) == 1:
                j = idx[0]
                if j != i:
                    acc += m[j] / np.linalg.norm(P[i] - P[j])
                continue
            R = P[i] - X
            d2 = float(R @ R)
            s = e / theta + np.linalg.norm(X - (lo + 0.5 * e))
            if d2 > s * s:
                d = math.sqrt(d2)
                acc += M / d + float(R @ Q @ R) / (2 * d ** 5)
            else:
                h = 0.5 * e
                for o in range(8):
                    stack.append((lo + h * np.array([o & 1, (o >> 1) & 1, (o >> 2) & 1], float), h))
        out.append(-acc)
    return np.array(out)


@pytest.mark.parametrize("theta", [0.4, 0.8])
def test_group_of_one_equals_textbook_bh(theta):
    g = random_amr(2, nbase=1, max_level=2, p_refine=0.6)
    t = OracleTree(g)
    t.walk(1, theta)
    phi = t.potential().ravel()
    x, y, z, m = t.cells()
    P = np.stack([x, y, z], 1)
    rng = np.random.default_rng(3)
    targets = rng.choice(t.ncells, 25, replace=False)
    ref = _textbook_bh(P, m, g.box_lo, g.box_size, theta, targets)
    assert np.max(np.abs(phi[targets] - ref) / np.abs(ref)) <= 1e-13


def _corner_mass_grid(levels=5):
    """Mass in one small block at a corner; every other leaf is empty."""
    def refine(L, lo, e):
        return bool(np.all(lo == 0.0))

    def dens(lo, h):
        r = np.zeros((lo.shape[0], 8, 8, 8))
        small = np.nonzero(h == h.min())[0]
        first = [i for i in small if np.all(lo[i] == 0.0)][0]
        rng = np.random.default_rng(9)
        r[first] = np.exp(rng.standard_normal((8, 8, 8)))
        return r
    return build_grid("corner_mass", 1, refine, levels, dens)


@pytest.mark.parametrize("order,slope", [(0, 2.0), (2, 3.0)])
def test_far_node_convergence_order(order, slope):
    g = _corner_mass_grid()
    t = OracleTree(g)
    t.walk(1, 1.0)
    phi = t.potential(order=order).ravel()
    x, y, z, m = t.cells()
    exact = t.direct()
    l = 1.0 / 32  # edge of the massive block
    mo = t.moments()
    root = int(np.nonzero(mo["key"] == np.uint64(0))[0][0])
    Xc = mo["X"][root]
    d = np.sqrt((x - Xc[0]) ** 2 + (y - Xc[1]) ** 2 + (z - Xc[2]) ** 2)
    rel = np.abs(phi - exact) / np.abs(exact)
    ds, es = [], []
    for lo_ in np.geomspace(4 * l, 24 * l, 8):
        sel = (d > lo_) & (d < lo_ * 1.15)
        if sel.sum() >= 5:
            ds.append(np.median(d[sel]))
            es.append(np.median(rel[sel]))
    fit = np.polyfit(np.log(ds), np.log(es), 1)[0]
    assert abs(-fit - slope) <= 0.25, (fit, ds, es)


def _cells_under(key, P, box_lo, box):
    d, ix, iy, iz = split_key(np.array([key]))
    e = box / float(1 << int(d[0]))
    lo = np.asarray(box_lo) + np.array([ix[0], iy[0], iz[0]], float) * e
    return np.nonzero(np.all((P > lo) & (P < lo + e), axis=1))[0]


def test_lists_cover_every_massive_cell_once():
    g = random_amr(31, nbase=2, max_level=2, p_refine=0.3, zero_fraction=0.15)
    t = OracleTree(g)
    w = t.walk(64, 0.6)
    x, y, z, m = t.cells()
    P = np.stack([x, y, z], 1)
    rng = np.random.default_rng(0)
    from oracle.oracle import make_key  # noqa: F401
    for gidx in rng.choice(t.n_groups(64), 12, replace=False):
        cover = np.zeros(t.ncells, np.int64)
        leaf, sub = divmod(int(gidx), 8)
        own = set()
        for q in range(64):
            mcode = sub * 64 + q
            i = sum(((mcode >> (3 * p)) & 1) << p for p in range(3))
            j = sum(((mcode >> (3 * p + 1)) & 1) << p for p in range(3))
            k = sum(((mcode >> (3 * p + 2)) & 1) << p for p in range(3))
            own.add(leaf * 512 + k * 64 + j * 8 + i)
        for key in w["far_keys"][w["far_off"][gidx]:w["far_off"][gidx + 1]]:
            cells = _cells_under(key, P, g.box_lo, g.box_size)
            assert not (set(cells.tolist()) & own), "an accepted node contains a group cell"
            cover[cells] += 1
        for key in w["near_keys"][w["near_off"][gidx]:w["near_off"][gidx + 1]]:
            cells = _cells_under(key, P, g.box_lo, g.box_size)
            assert len(cells) == 8
            cover[cells] += 1
        massive = m > 0
        assert np.all(cover[massive] == 1)
        assert np.all(cover <= 1)


def test_error_grows_with_theta_percent_level_at_one():
    g = uniform_sphere(nbase=4)
    t = OracleTree(g)
    d = t.direct()
    errs = []
    for th in (0.25, 0.5, 0.75, 1.0):
        t.walk(64, th)
        for order in (0, 2):
            phi = t.potential(order=order).ravel()
            errs.append((th, order, float(np.max(np.abs(phi - d) / np.abs(d)))))
    mono = [e for th, o, e in errs if o == 0]
    quad = [e for th, o, e in errs if o == 2]
    assert all(a < b for a, b in zip(mono, mono[1:]))
    assert all(a < b for a, b in zip(quad, quad[1:]))
    # theta = 1, monopole only: percent-level error (section 2)
    assert 1e-3 < mono[-1] < 3e-2
    # the quadrupole improves every theta
    assert all(q < mo for q, mo in zip(quad, mono))


def test_group_subset_solve_equals_full_solve():
    g = random_amr(21, nbase=2, max_level=3, zero_fraction=0.1)
    t = OracleTree(g)
    w = t.walk(64, 0.6)
    phi = t.potential().reshape(-1)
    gs = np.array([0, 5, 17, 100, t.n_groups(64) - 1])
    ps, cs = t.solve_groups(gs, theta=0.6)
    for q, gi in enumerate(gs):
        leaf, sub = divmod(int(gi), 8)
        mm = sub * 64 + np.arange(64)
        i = sum(((mm >> (3 * p)) & 1) << p for p in range(3))
        j = sum(((mm >> (3 * p + 1)) & 1) << p for p in range(3))
        k = sum(((mm >> (3 * p + 2)) & 1) << p for p in range(3))
        assert np.array_equal(ps[q], phi[leaf * 512 + k * 64 + j * 8 + i])
        assert cs[q, 1] == w["n_far"][gi] and cs[q, 2] == w["n_near"][gi] and cs[q, 0] == w["visited"][gi]
