"""Pins of the oracle's periodic Barnes-Hut (O10) and of what it is built from:
the Hessian of the Ewald smooth part (O9) and the second-moment trace S of the
nodes (O3).  None of these re-types the oracle's formulas:

* Hessian of D: central differences of the gradient; its trace is the
  Laplacian 4 pi / L^3 of the neutralising background; independent of the
  splitting constant (which moves points between the series and the closed
  form of the image-0 term);
* S = sum m |r - X|^2: the closed form M h^2 (n^2 - 1) / 4 of an n^3 lattice of
  equal masses, and the parallel-axis rule between every node and its children;
* a single far node's term converges to the exact sum of its cells' periodic
  Green's functions, each added part (quadrupole, Q:H / 6, the S term)
  shrinking the error, and the full term's error falls like (l / d)^3;
* with every node opened (tiny theta) the periodic walk and sum equal the
  exact periodic direct sum;
* translating the density by half the box (a permutation of the root's
  children) permutes the periodic potential;
* the error against the exact periodic direct sum falls with theta and, at
  theta = 0.5, is within a few times that of the isolated method on the same
  grid (the periodic potential has zero mean and is much smaller than the
  isolated one, so errors are compared in absolute terms).

Error metric: periodic potentials have zero mean (the neutralising
background), so cell-wise relative errors are ill-conditioned; the periodic
metric is ||phi - phi_ref|| / ||phi_ref|| over the sampled cells.
"""
import numpy as np
import pytest

from amr_inputs import random_amr, single_block, uniform_sphere
from oracle import OracleTree
from oracle.oracle import ewald, ewald_hessian, make_key, split_key

FOUR_PI = 4.0 * np.pi


def _points(n, seed, lo=0.02, hi=0.45):
    rng = np.random.default_rng(seed)
    return rng.uniform(lo, hi, (n, 3)) * rng.choice([-1.0, 1.0], (n, 3))


def test_hessian_is_the_derivative_of_the_gradient():
    p = _points(12, 5)
    D, g, H = ewald_hessian(p)
    D0, g0 = ewald(p)
    assert np.array_equal(D, D0) and np.array_equal(g, g0)
    step = 1e-5
    cols = {0: [0, 3, 4], 1: [3, 1, 5], 2: [4, 5, 2]}
    for k in range(3):
        e = np.zeros(3)
        e[k] = step
        _, gp, _ = ewald_hessian(p + e)
        _, gm, _ = ewald_hessian(p - e)
        assert np.max(np.abs((gp - gm) / (2 * step) - H[:, cols[k]])) <= 1e-7
    assert np.max(np.abs(H[:, 0] + H[:, 1] + H[:, 2] - FOUR_PI)) <= 1e-11


def test_hessian_does_not_depend_on_the_splitting_constant():
    # |r| ~ 0.02..0.06: a r straddles 0.1, so both forms of the image-0 term are used
    p = _points(16, 6, lo=0.01, hi=0.035)
    _, ga, Ha = ewald_hessian(p, alpha=2.0)
    _, gb, Hb = ewald_hessian(p, alpha=3.5, nreal=4, nrecip=7)
    assert np.max(np.abs(ga - gb)) <= 1e-13
    assert np.max(np.abs(Ha - Hb)) <= 1e-12 * np.max(np.abs(Ha))


def test_trace_moment_closed_form_on_a_uniform_block():
    g = single_block(seed=0, sigma=0.0)
    mo = OracleTree(g).moments()
    h = g.box_size / 8
    n = np.rint(mo["edge"] / h)
    ok = mo["M"] > 0
    ref = mo["M"][ok] * h * h * (n[ok] ** 2 - 1) / 4
    assert np.max(np.abs(mo["S"][ok] - ref)) <= 1e-14 * np.max(np.abs(ref))


def test_trace_moment_parallel_axis_rule():
    g = random_amr(63, nbase=2, max_level=2, p_refine=0.3, zero_fraction=0.1)
    mo = OracleTree(g).moments()
    idx = {int(k): n for n, k in enumerate(mo["key"])}
    d, ix, iy, iz = split_key(mo["key"])
    checked = 0
    for n in np.nonzero((mo["bottom"] == 0) & (mo["M"] > 0))[0]:
        kids = [idx.get(int(make_key(d[n] + 1, 2 * ix[n] + (o & 1), 2 * iy[n] + ((o >> 1) & 1),
                                     2 * iz[n] + ((o >> 2) & 1))), -1) for o in range(8)]
        kids = [c for c in kids if c >= 0]
        s = sum(mo["S"][c] + mo["M"][c] * np.sum((mo["X"][c] - mo["X"][n]) ** 2) for c in kids)
        assert abs(s - mo["S"][n]) <= 1e-12 * mo["S"][n]
        checked += 1
    assert checked > 20


def test_far_term_converges_to_the_cells_and_each_part_helps():
    g = random_amr(61, nbase=2, max_level=1, p_refine=0.3, zero_fraction=0.1)
    t = OracleTree(g)
    mo = t.moments()
    x, y, z, m = t.cells()
    P = np.stack([x, y, z], 1)
    L = g.box_size
    errs = []
    for n in np.nonzero(np.isclose(mo["edge"], L / 8) & (mo["M"] > 0))[0][:6]:
        inside = np.all(np.abs(P - mo["centre"][n]) < mo["edge"][n] / 2, axis=1)
        for off in ([0.3, 0.1, 0.0], [0.2, 0.2, 0.2], [0.0, 0.35, 0.1], [0.42, 0.0, 0.0]):
            p = mo["X"][n] + np.array(off) * L
            parts = t.node_far_periodic(n, p)
            R = p - P[inside]
            R -= L * np.rint(R / L)
            D, _ = ewald(R, L)
            exact = np.sum(m[inside] * (1.0 / np.linalg.norm(R, axis=1) + D))
            dist = np.linalg.norm(np.array(off) * L)
            scale = mo["M"][n] / dist
            method = parts.sum()
            # the smooth part alone: M D(R) (the first part less M / |R|), then + the S term, + the Q:H term
            d_exact = np.sum(m[inside] * D)
            d_mono = parts[0] - mo["M"][n] / dist
            errs.append([abs(parts[0] - exact) / scale, abs(parts[0] + parts[1] - exact) / scale,
                         abs(method - exact) / scale, abs(d_mono - d_exact) / abs(d_exact),
                         abs(d_mono + parts[3] - d_exact) / abs(d_exact),
                         abs(d_mono + parts[3] + parts[2] - d_exact) / abs(d_exact)])
            # third order: l / d <= 0.42 here
            assert errs[-1][2] <= 0.2 * (mo["edge"][n] / dist) ** 3
    e = np.array(errs)
    # mean errors: monopole > + quadrupole > + Q:H/6 and S (the method's far term)
    assert e[:, 0].mean() > e[:, 1].mean() > 2 * e[:, 2].mean()
    # the smooth part's own expansion: the S term cuts its error tenfold, the Q:H term again
    assert e[:, 3].mean() > 10 * e[:, 4].mean() and e[:, 4].mean() > 2 * e[:, 5].mean()


def _group_cells(gi):
    mm = np.arange(64) + (gi % 8) * 64
    i = sum(((mm >> (3 * p)) & 1) << p for p in range(3))
    j = sum(((mm >> (3 * p + 1)) & 1) << p for p in range(3))
    k = sum(((mm >> (3 * p + 2)) & 1) << p for p in range(3))
    return (gi // 8) * 512 + k * 64 + j * 8 + i


@pytest.fixture(scope="module")
def small():
    g = random_amr(61, nbase=2, max_level=1, p_refine=0.3, zero_fraction=0.1)
    t = OracleTree(g)
    t.moments()
    ng = t.n_groups(64)
    gs = np.array([0, ng // 3, ng - 1])
    tg = np.concatenate([_group_cells(q) for q in gs])
    return g, t, gs, t.direct_periodic(tg)


def test_every_node_opened_gives_the_periodic_direct_sum(small):
    g, t, gs, ref = small
    phi, counts = t.solve_groups_periodic(gs, theta=0.02)
    assert np.all(counts[:, 1] == 0)
    assert np.max(np.abs(phi.ravel() - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_error_falls_with_theta_and_matches_the_isolated_method(small):
    g, t, gs, ref = small
    e = []
    for th in (0.4, 0.5, 0.8):
        phi, _ = t.solve_groups_periodic(gs, theta=th)
        e.append(np.linalg.norm(phi.ravel() - ref))
    assert e[0] < e[1] < e[2]
    # absolute error at theta = 0.5 within a few times that of the isolated method on the same grid (the
    # nodes near the half-box planes also carry the neighbouring image in D, whose next term is left out)
    iso, _ = t.solve_groups(gs, theta=0.5)
    iso_ref = t.direct(np.concatenate([_group_cells(q) for q in gs]))
    assert e[1] <= 4.0 * np.linalg.norm(iso.ravel() - iso_ref)


def test_half_box_translation_permutes_the_potential():
    g = random_amr(64, nbase=2, max_level=0)  # 2^3 base blocks: a shift by one block permutes the root's children
    t = OracleTree(g)
    lo = np.asarray(g.lo)
    e = g.box_size / 2
    partner = [int(np.nonzero(np.all(np.isclose(lo, (lo[b] + [e, 0, 0]) % g.box_size), axis=1))[0][0])
               for b in range(g.nleaf)]
    rho2 = np.empty_like(g.rho)
    for b in range(g.nleaf):
        rho2[partner[b]] = g.rho[b]
    t2 = OracleTree(g)
    t2.set_density(rho2)
    gs = np.array([3, 20, 45])
    p1, c1 = t.solve_groups_periodic(gs, theta=0.7, tau=1e-12)
    moved = np.array([partner[q // 8] * 8 + q % 8 for q in gs])
    p2, c2 = t2.solve_groups_periodic(moved, theta=0.7, tau=1e-12)
    ok = (c1[:, 3] == 0) & (c2[:, 3] == 0)
    assert ok.sum() >= 2
    assert np.array_equal(c1[ok, :3], c2[ok, :3])
    assert np.max(np.abs(p1[ok] - p2[ok])) <= 1e-12 * np.max(np.abs(p1))


def test_accuracy_at_theta_half_on_a_sphere():
    """Absolute accuracy pin: on the uniform sphere of the opening configuration
    (16^3 cells, sixteen groups spread over the grid), the periodic walk and sum
    at theta = 0.5 come within 5e-4 of the exact periodic direct sum in the
    normalised norm.  That is a third of the maximum error the paper reports
    for its isolated method at theta = 0.5 (1.4e-3, Fig. Errors), and the
    quadrupole keeps this method's own isolated error at 5e-6 on the same
    cells; the periodic error is larger because the expansion of D is cut at
    second order near the half-box planes (measured 1.3e-4)."""
    g = uniform_sphere(nbase=2)
    t = OracleTree(g)
    t.moments()
    gs = np.unique(np.linspace(0, t.n_groups(64) - 1, 16).astype(int))
    ref = t.direct_periodic(np.concatenate([_group_cells(q) for q in gs]))
    phi, counts = t.solve_groups_periodic(gs, theta=0.5)
    assert counts[:, 1].sum() > 0  # far nodes were accepted
    err = np.linalg.norm(phi.ravel() - ref) / np.linalg.norm(ref)
    assert err <= 5e-4, err
