"""Pins of the oracle's node moments (O3).

The oracle computes every node straight from its own cells.  These checks use
routes that do not go through its code: cells selected by geometry from the
node key, the parallel-axis combination of children, symmetry, and trace.
"""
import numpy as np

from amr_inputs import random_amr, uniform_sphere
from oracle import OracleTree
from oracle.oracle import split_key


def _node_bounds(key, box_lo, box):
    d, ix, iy, iz = split_key(np.array([key]))
    e = box / float(1 << int(d[0]))
    lo = np.asarray(box_lo) + np.array([ix[0], iy[0], iz[0]], float) * e
    return lo, lo + e


def test_moments_from_geometry_selection():
    g = random_amr(5, nbase=2, max_level=2, p_refine=0.3, zero_fraction=0.1)
    t = OracleTree(g)
    mo = t.moments()
    x, y, z, m = t.cells()
    P = np.stack([x, y, z], 1)
    rng = np.random.default_rng(1)
    for n in rng.choice(t.nnodes, 60, replace=False):
        lo, hi = _node_bounds(mo["key"][n], g.box_lo, g.box_size)
        sel = np.all((P > lo) & (P < hi), axis=1)
        M = m[sel].sum()
        assert np.isclose(mo["M"][n], M, rtol=1e-13, atol=0)
        if M == 0:
            assert np.allclose(mo["X"][n], 0.5 * (lo + hi)) and np.all(mo["Q"][n] == 0) and mo["delta"][n] == 0
            continue
        X = (m[sel, None] * P[sel]).sum(0) / M
        D = P[sel] - X
        r2 = (D * D).sum(1)
        Q = np.array([np.sum(m[sel] * (3 * D[:, 0] ** 2 - r2)), np.sum(m[sel] * (3 * D[:, 1] ** 2 - r2)),
                      np.sum(m[sel] * (3 * D[:, 2] ** 2 - r2)), np.sum(m[sel] * 3 * D[:, 0] * D[:, 1]),
                      np.sum(m[sel] * 3 * D[:, 0] * D[:, 2]), np.sum(m[sel] * 3 * D[:, 1] * D[:, 2])])
        l = hi[0] - lo[0]
        assert np.allclose(mo["X"][n], X, rtol=0, atol=2e-15)
        assert np.allclose(mo["Q"][n], Q, rtol=0, atol=1e-12 * M * l * l)
        assert np.isclose(mo["delta"][n], np.linalg.norm(X - 0.5 * (lo + hi)), rtol=0, atol=2e-15)


def test_parallel_axis_consistency_and_trace():
    g = random_amr(8, nbase=2, max_level=2, p_refine=0.35)
    t = OracleTree(g)
    mo = t.moments()
    key = mo["key"]
    index = {int(k): i for i, k in enumerate(key)}
    d, ix, iy, iz = split_key(key)
    root = index[int(np.uint64(0))]
    assert np.isclose(mo["M"][root], (g.rho * g.cell_volumes()[:, None, None, None]).sum(), rtol=1e-14)
    checked = 0
    for n in range(t.nnodes):
        M, X, Q = mo["M"][n], mo["X"][n], mo["Q"][n]
        l = mo["edge"][n]
        # traceless
        assert abs(Q[0] + Q[1] + Q[2]) <= 1e-13 * M * l * l + 1e-300
        if mo["bottom"][n]:
            continue
        kids = []
        for o in range(8):
            ck = (np.uint64(d[n] + 1) << np.uint64(57)) | (np.uint64(2 * ix[n] + (o & 1)) << np.uint64(38)) | \
                 (np.uint64(2 * iy[n] + ((o >> 1) & 1)) << np.uint64(19)) | np.uint64(2 * iz[n] + ((o >> 2) & 1))
            kids.append(index[int(ck)])
        Mc = mo["M"][kids]
        assert np.isclose(M, Mc.sum(), rtol=1e-14)
        if M == 0:
            continue
        Xp = (Mc[:, None] * mo["X"][kids]).sum(0) / M
        assert np.allclose(X, Xp, rtol=0, atol=2e-15)
        Dd = mo["X"][kids] - X
        r2 = (Dd * Dd).sum(1)
        shift = np.stack([Mc * (3 * Dd[:, 0] ** 2 - r2), Mc * (3 * Dd[:, 1] ** 2 - r2), Mc * (3 * Dd[:, 2] ** 2 - r2),
                          Mc * 3 * Dd[:, 0] * Dd[:, 1], Mc * 3 * Dd[:, 0] * Dd[:, 2], Mc * 3 * Dd[:, 1] * Dd[:, 2]], 1)
        Qp = (mo["Q"][kids] + shift).sum(0)
        assert np.allclose(Q, Qp, rtol=0, atol=1e-12 * M * l * l)
        checked += 1
    assert checked > 100


def test_uniform_block_nodes_have_no_quadrupole_and_centred_com():
    g = uniform_sphere(nbase=2, rho_in=1.0, rho_out=1.0)  # uniform density everywhere
    t = OracleTree(g)
    mo = t.moments()
    for n in range(t.nnodes):
        l = mo["edge"][n]
        assert np.all(np.abs(mo["Q"][n]) <= 1e-13 * mo["M"][n] * l * l)
        assert mo["delta"][n] <= 1e-14 * l
