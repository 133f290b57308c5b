"""Pins of the oracle's group-cube opening test (O5b, the paper's test between a
node and a whole region, Fig. opening_angles2) and of the monopole-only sum.

* O5b lists equal those of an independent Python walk over the oracle's node
  table, which measures the distance from a node's centre of mass to the
  group's cube with a numpy clamp (groups the oracle flags as marginal aside);
* O5b is the stricter test (the cube holds every cell centre): every node it
  accepts is, or lies below, a node that the per-cell vote accepts;
* every massive cell is covered exactly once per group under O5b too;
* monopole-only sums (order 0) are what the convergence-order pin of
  test_oracle_bh exercises; here: order 0 equals order 2 on a grid whose
  nodes all have Q = 0 (a uniform single block), and differs elsewhere.
"""
import numpy as np
import pytest

from amr_inputs import random_amr, single_block
from oracle import OracleTree
from oracle.oracle import make_key, split_key


def _group_cells(leaf, sub):
    m = sub * 64 + np.arange(64)
    i = sum(((m >> (3 * p)) & 1) << p for p in range(3))
    j = sum(((m >> (3 * p + 1)) & 1) << p for p in range(3))
    k = sum(((m >> (3 * p + 2)) & 1) << p for p in range(3))
    return leaf * 512 + k * 64 + j * 8 + i


def _python_cube_walk(t, g, theta):
    """Recursive walk over the oracle's node table with a numpy point-to-cube distance."""
    mo = t.moments()
    idx = {int(k): n for n, k in enumerate(mo["key"])}
    x, y, z, _ = t.cells()
    P = np.stack([x, y, z], 1)
    leaf, sub = divmod(g, 8)
    cells = _group_cells(leaf, sub)
    h = float(mo["edge"][idx[int(_leaf_block_key(t, leaf))]]) / 8.0
    lo = P[cells].min(0) - 0.5 * h
    hi = P[cells].max(0) + 0.5 * h
    far, near = [], []

    def visit(key):
        n = idx[key]
        if mo["M"][n] == 0.0:
            return
        X = mo["X"][n]
        gap = X - np.clip(X, lo, hi)
        s = mo["edge"][n] / theta + mo["delta"][n]
        if gap @ gap > s * s:
            far.append(key)
        elif mo["bottom"][n]:
            near.append(key)
        else:
            d, ix, iy, iz = (int(v[0]) for v in split_key(np.array([key], np.uint64)))
            for o in range(8):
                ck = int(make_key(d + 1, 2 * ix + (o & 1), 2 * iy + ((o >> 1) & 1), 2 * iz + ((o >> 2) & 1)))
                if ck in idx:
                    visit(ck)

    visit(int(make_key(0, 0, 0, 0)))
    return sorted(far), sorted(near)


def _leaf_block_key(t, leaf):
    """key of the leaf block holding canonical leaf `leaf` (the parent of its octants)."""
    x, y, z, _ = t.cells()
    c = leaf * 512
    mo = t.moments()
    # the block is the deepest non-bottom node of edge 8 h containing the first cell
    best = None
    for n in np.nonzero(mo["bottom"] == 0)[0]:
        ctr, e = mo["centre"][n], mo["edge"][n]
        p = np.array([x[c], y[c], z[c]])
        if np.all(np.abs(p - ctr) < e / 2) and (best is None or e < mo["edge"][best]):
            best = n
    # `best` is an octant (4^3 cells); its parent is the block
    d, ix, iy, iz = (int(v[0]) for v in split_key(mo["key"][best:best + 1]))
    return make_key(d - 1, ix >> 1, iy >> 1, iz >> 1)


@pytest.mark.parametrize("theta", [0.5, 0.9])
def test_cube_walk_equals_python_walk(theta):
    g = random_amr(51, nbase=2, max_level=2, p_refine=0.4, zero_fraction=0.1)
    t = OracleTree(g)
    w = t.walk(64, theta, tau=1e-12, mac=1)
    rng = np.random.default_rng(1)
    for gi in rng.choice(t.n_groups(64), min(10, t.n_groups(64)), replace=False):
        if w["marginal"][gi]:
            continue
        far, near = _python_cube_walk(t, int(gi), theta)
        assert sorted(w["far_keys"][w["far_off"][gi]:w["far_off"][gi + 1]].tolist()) == far
        assert sorted(w["near_keys"][w["near_off"][gi]:w["near_off"][gi + 1]].tolist()) == near


def _ancestors(key):
    d, ix, iy, iz = (int(v[0]) for v in split_key(np.array([key], np.uint64)))
    out = []
    while d > 0:
        d, ix, iy, iz = d - 1, ix >> 1, iy >> 1, iz >> 1
        out.append(int(make_key(d, ix, iy, iz)))
    return out


def test_cube_test_is_stricter_than_cell_vote():
    g = random_amr(52, nbase=2, max_level=2, p_refine=0.3, zero_fraction=0.1)
    t = OracleTree(g)
    cube = t.walk(64, 0.7, mac=1)
    cell = t.walk(64, 0.7, mac=0)
    for gi in range(0, t.n_groups(64), 7):
        accepted = set(cell["far_keys"][cell["far_off"][gi]:cell["far_off"][gi + 1]].tolist())
        for k in cube["far_keys"][cube["far_off"][gi]:cube["far_off"][gi + 1]].tolist():
            assert k in accepted or any(a in accepted for a in _ancestors(k))
        assert cube["n_far"][gi] + cube["n_near"][gi] >= 1


def test_cube_walk_covers_every_massive_cell_once():
    g = random_amr(53, nbase=2, max_level=2, p_refine=0.3, zero_fraction=0.15)
    t = OracleTree(g)
    w = t.walk(64, 0.8, mac=1)
    x, y, z, m = t.cells()
    P = np.stack([x, y, z], 1)
    for gi in np.random.default_rng(2).choice(t.n_groups(64), 8, replace=False):
        cover = np.zeros(t.ncells, np.int64)
        for key in np.concatenate([w["far_keys"][w["far_off"][gi]:w["far_off"][gi + 1]],
                                   w["near_keys"][w["near_off"][gi]:w["near_off"][gi + 1]]]):
            d, ix, iy, iz = split_key(np.array([key]))
            e = g.box_size / float(1 << int(d[0]))
            lo = np.asarray(g.box_lo) + np.array([ix[0], iy[0], iz[0]], float) * e
            cover[np.all((P > lo) & (P < lo + e), axis=1)] += 1
        assert np.all(cover[m > 0] == 1)


def test_monopole_only_order():
    g = single_block(seed=0, sigma=0.0)  # uniform block: every node has Q = 0
    t = OracleTree(g)
    t.walk(64, 0.9)
    assert np.array_equal(t.potential(order=0), t.potential(order=2))
    g2 = random_amr(54, nbase=2, max_level=1)
    t2 = OracleTree(g2)
    t2.walk(64, 0.9)
    assert not np.array_equal(t2.potential(order=0), t2.potential(order=2))
