"""Pins of the oracle's periodic Green's function (O9, appendix "Periodic
boundaries": Ewald's split into short- and long-range sums) and of the exact
periodic direct sum.

* D = psi - 1/r does not depend on the splitting constant;
* psi(r) = D(r) + 1/|r| is periodic in every direction;
* away from the lattice points, Laplacian(psi) = 4 pi / L^3 (the neutralising
  background), by finite differences;
* grad D matches central finite differences of D; D is even in each axis and
  symmetric under axis permutations;
* the self term D(0) is the simple cubic lattice constant -2.8372974794806/L;
* a uniform lattice of cells in a periodic box has the same potential at every
  cell, +2.8372974794806 G m / h (the constant at the cell spacing);
* shifting a density field by one base block (periodically) permutes the
  potential accordingly.
"""
import numpy as np
import pytest

from amr_inputs import random_amr, single_block
from oracle import OracleTree
from oracle.oracle import ewald

LATTICE = -2.8372974794806


def _points(n, seed, L=1.0, lo=0.05, hi=0.45):
    rng = np.random.default_rng(seed)
    p = rng.uniform(lo, hi, (n, 3)) * L
    return p * rng.choice([-1.0, 1.0], (n, 3))


def test_splitting_constant_does_not_matter():
    p = _points(20, 0)
    Da, ga = ewald(p, alpha=2.0)
    Db, gb = ewald(p, alpha=3.5, nreal=4, nrecip=7)
    assert np.max(np.abs(Da - Db)) <= 1e-13
    assert np.max(np.abs(ga - gb)) <= 1e-12


@pytest.mark.parametrize("L", [1.0, 2.0])
def test_self_term_is_the_cubic_lattice_constant(L):
    D, g = ewald(np.zeros((1, 3)), L=L)
    assert abs(D[0] - LATTICE / L) <= 1e-12 / L
    assert np.max(np.abs(g)) <= 1e-13


def test_psi_is_periodic():
    p = _points(10, 1)
    for k in range(3):
        e = np.zeros(3)
        e[k] = 1.0
        D0, _ = ewald(p)
        D1, _ = ewald(p + e)
        psi0 = D0 + 1.0 / np.linalg.norm(p, axis=1)
        psi1 = D1 + 1.0 / np.linalg.norm(p + e, axis=1)
        assert np.max(np.abs(psi0 - psi1)) <= 1e-12


def test_laplacian_is_the_background_and_gradient_is_consistent():
    p = _points(8, 2)
    step = 1e-3
    D0, g0 = ewald(p)
    lap = -6.0 * D0
    for k in range(3):
        e = np.zeros(3)
        e[k] = step
        Dp, _ = ewald(p + e)
        Dm, _ = ewald(p - e)
        lap += Dp + Dm
        gp, _ = ewald(p + e * 0.1)
        gm, _ = ewald(p - e * 0.1)
        assert np.max(np.abs((gp - gm) / (0.2 * step) - g0[:, k])) <= 1e-7
    lap /= step * step
    # Laplacian(1/r) = 0 away from 0, so Laplacian(D) = Laplacian(psi) = 4 pi / L^3
    assert np.max(np.abs(lap - 4.0 * np.pi)) <= 1e-4


def test_symmetries():
    p = _points(6, 3)
    D0, _ = ewald(p)
    D1, _ = ewald(p * np.array([-1.0, 1.0, 1.0]))
    D2, _ = ewald(p[:, [1, 2, 0]])
    assert np.max(np.abs(D0 - D1)) <= 1e-13 and np.max(np.abs(D0 - D2)) <= 1e-13


def test_uniform_lattice_in_a_periodic_box():
    g = single_block(seed=0, sigma=0.0)
    t = OracleTree(g)
    x, y, z, m = t.cells()
    h = g.box_size / 8
    phi = t.direct_periodic(np.array([0, 73, 300, 511]))
    assert np.max(np.abs(phi - (-LATTICE) * m[0] / h)) <= 1e-12 * abs(LATTICE * m[0] / h)


def test_shift_by_one_block_permutes_the_potential():
    g = random_amr(62, nbase=2, max_level=0)  # 2^3 base blocks, no refinement
    t = OracleTree(g)
    # blocks are in canonical order; find the block one base step along x for each block
    lo = np.asarray(g.lo)
    e = g.box_size / 2
    partner = [int(np.nonzero(np.all(np.isclose(lo, (lo[b] + [e, 0, 0]) % g.box_size), axis=1))[0][0])
               for b in range(g.nleaf)]
    rho2 = np.empty_like(g.rho)
    for b in range(g.nleaf):
        rho2[partner[b]] = g.rho[b]
    tg = np.array([5, 600, 3000])
    phi1 = t.direct_periodic(tg)
    t2 = OracleTree(g)
    t2.set_density(rho2)
    moved = np.array([partner[c // 512] * 512 + c % 512 for c in tg])
    phi2 = t2.direct_periodic(moved)
    assert np.max(np.abs(phi1 - phi2) / np.abs(phi1)) <= 1e-12
