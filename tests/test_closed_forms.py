"""Closed forms that pin the physics the oracle's direct sum must reproduce.

* the MacLaurin formulas of section "Accuracy with the MacLaurin Sphere", as
  corrected (interior A3 sign, exterior 1/(a1 e) factor), against the general
  homogeneous-ellipsoid integral -- and the printed forms shown to fail it;
* uniform sphere and homogeneous prism against quadrature / Poisson's equation;
* the oracle's direct sum converging to these continuum potentials as the
  mesh is refined (discretisation-limited agreement, as in the paper's
  direct-sum comparison).
"""
import math

import numpy as np
import pytest

from amr_inputs import maclaurin_spheroid, plummer_sphere, uniform_sphere
from oracle import OracleTree
from oracle.closed_forms import (ellipsoid_potential_integral, maclaurin_A, maclaurin_potential, prism_potential,
                                 plummer_potential, sphere_potential)

E, A1AX = 0.9, 0.25
POINTS = [(0.0, 0.0, 0.0), (0.1, 0.05, 0.03), (0.2, -0.1, 0.02), (0.0, 0.0, 0.1), (0.3, 0.0, 0.0),
          (0.0, 0.0, 0.2), (0.2, 0.1, 0.15), (-0.4, 0.3, -0.2), (1.0, 1.0, 1.0), (0.26, 0.0, 0.0)]


@pytest.mark.parametrize("p", POINTS)
def test_maclaurin_closed_form_matches_ellipsoid_integral(p):
    a3 = A1AX * math.sqrt(1 - E * E)
    ref = ellipsoid_potential_integral(*p, (A1AX, A1AX, a3), rho=1.0)
    got = float(maclaurin_potential(*p, E, A1AX, rho=1.0))
    assert got == pytest.approx(ref, rel=1e-10)


def test_printed_maclaurin_forms_fail_the_integral():
    """The printed interior sign and the printed exterior bracket are not the potential."""
    a3 = A1AX * math.sqrt(1 - E * E)
    A1, A3 = maclaurin_A(E)
    # printed interior bracket (positive convention), negated to phi < 0
    x, y, z = 0.1, 0.05, 0.03
    printed_in = -math.pi * (2 * A1 * A1AX ** 2 - A1 * (x * x + y * y) - A3 * (a3 * a3 - z * z))
    ref = ellipsoid_potential_integral(x, y, z, (A1AX, A1AX, a3), 1.0)
    assert abs(printed_in - ref) > 1e-2 * abs(ref)
    # printed exterior bracket without 1/(a1 e)
    x, y, z = 0.3, 0.0, 0.1
    R2, z2 = x * x + y * y, z * z
    b = A1AX ** 2 + a3 ** 2 - R2 - z2
    c = A1AX ** 2 * a3 ** 2 - R2 * a3 ** 2 - z2 * A1AX ** 2
    lam = 0.5 * (-b + math.sqrt(b * b - 4 * c))
    h = A1AX * E / math.sqrt(a3 * a3 + lam)
    printed_out = -(2 * a3 / E ** 2) * math.pi * (A1AX * E * math.atan(h) - 0.5 * (
        R2 * (math.atan(h) - h / (1 + h * h)) + 2 * z2 * (h - math.atan(h))))
    ref = ellipsoid_potential_integral(x, y, z, (A1AX, A1AX, a3), 1.0)
    assert abs(printed_out - ref) > 1e-2 * abs(ref)
    # identity 2 A1 + A3 = 2 (Poisson's equation inside)
    assert 2 * A1 + A3 == pytest.approx(2.0, rel=1e-14)


def test_maclaurin_continuity_and_far_field():
    a3 = A1AX * math.sqrt(1 - E * E)
    for th in np.linspace(0.1, 3.0, 7):
        px, pz = A1AX * math.sin(th), a3 * math.cos(th)
        inn = maclaurin_potential(px * (1 - 1e-9), 0, pz * (1 - 1e-9), E, A1AX, 1.0)
        out = maclaurin_potential(px * (1 + 1e-9), 0, pz * (1 + 1e-9), E, A1AX, 1.0)
        assert float(inn) == pytest.approx(float(out), rel=1e-7)
    M = 4 / 3 * math.pi * A1AX * A1AX * a3
    r = 200.0
    assert float(maclaurin_potential(r, 0, 0, E, A1AX, 1.0)) == pytest.approx(-M / r, rel=1e-5)


def test_sphere_closed_form_matches_integral():
    R = 0.4
    for p in [(0, 0, 0), (0.1, 0.2, 0.1), (0.3, 0.3, 0.3), (1, 0, 0)]:
        r = math.sqrt(sum(v * v for v in p))
        ref = ellipsoid_potential_integral(*p, (R, R, R), 1.0)
        assert float(sphere_potential(r, R, 1.0)) == pytest.approx(ref, rel=1e-10)


def _gauss_prism(p, lo, hi, n=48):
    xg, wg = np.polynomial.legendre.leggauss(n)
    pts = [0.5 * (hi[d] - lo[d]) * xg + 0.5 * (hi[d] + lo[d]) for d in range(3)]
    ws = [0.5 * (hi[d] - lo[d]) * wg for d in range(3)]
    X, Y, Z = np.meshgrid(*pts, indexing="ij")
    W = ws[0][:, None, None] * ws[1][None, :, None] * ws[2][None, None, :]
    r = np.sqrt((X - p[0]) ** 2 + (Y - p[1]) ** 2 + (Z - p[2]) ** 2)
    return -np.sum(W / r)


def test_prism_closed_form():
    lo, hi = (0.0, 0.0, 0.0), (1.0, 0.5, 0.25)
    for p in [(2.0, 0.3, 0.1), (0.5, 1.5, -0.5), (-1.0, -1.0, 2.0)]:
        assert float(prism_potential(*p, lo, hi, 1.0)) == pytest.approx(_gauss_prism(p, lo, hi), rel=1e-10)
    # far field -> -G M / r
    M = 1.0 * 0.5 * 0.25
    c = np.array([0.5, 0.25, 0.125])
    p = c + np.array([300.0, 100.0, -50.0])
    assert float(prism_potential(*p, lo, hi, 1.0)) == pytest.approx(-M / np.linalg.norm(p - c), rel=1e-6)
    # Poisson's equation inside: laplacian = 4 pi G rho
    q = np.array([0.3, 0.2, 0.1])
    hstep = 1e-3
    lap = 0.0
    for d in range(3):
        e = np.zeros(3)
        e[d] = hstep
        lap += (float(prism_potential(*(q + e), lo, hi, 1.0)) - 2 * float(prism_potential(*q, lo, hi, 1.0))
                + float(prism_potential(*(q - e), lo, hi, 1.0))) / hstep ** 2
    assert lap == pytest.approx(4 * math.pi, rel=1e-4)


def _sample_targets(n, count, seed=0):
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(n, size=min(count, n), replace=False))


def test_direct_sum_converges_to_sphere_potential():
    """Uniform sphere in a low-density box: sphere (rho_in - rho_out) + prism (rho_out)."""
    errs = []
    for nbase in (2, 4, 8):
        g = uniform_sphere(nbase=nbase)
        t = OracleTree(g)
        tg = _sample_targets(t.ncells, 300, seed=nbase)
        phi = t.direct(tg)
        x, y, z, _ = t.cells()
        c = np.array(g.meta["centre"])
        r = np.sqrt((x[tg] - c[0]) ** 2 + (y[tg] - c[1]) ** 2 + (z[tg] - c[2]) ** 2)
        exact = sphere_potential(r, g.meta["radius"], g.meta["rho_in"] - g.meta["rho_out"]) + prism_potential(
            x[tg], y[tg], z[tg], (0, 0, 0), (1, 1, 1), g.meta["rho_out"])
        errs.append(float(np.sqrt(np.mean(((phi - exact) / exact) ** 2))))
    # discretisation-limited: the error falls steadily under refinement
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 2e-3
    assert errs[1] / errs[2] > 1.5


def test_direct_sum_converges_to_maclaurin():
    errs = []
    for lev in (0, 1, 2):
        g = maclaurin_spheroid(max_level=lev, nbase=4)
        t = OracleTree(g)
        tg = _sample_targets(t.ncells, 200, seed=lev)
        phi = t.direct(tg)
        x, y, z, _ = t.cells()
        c = np.array(g.meta["centre"])
        exact = maclaurin_potential(x[tg] - c[0], y[tg] - c[1], z[tg] - c[2], g.meta["e"], g.meta["a1"],
                                    g.meta["rho_in"] - g.meta["rho_out"]) + prism_potential(
            x[tg], y[tg], z[tg], (0, 0, 0), (1, 1, 1), g.meta["rho_out"])
        errs.append(float(np.max(np.abs((phi - exact) / exact))))
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 1e-2


def test_direct_sum_converges_to_plummer_potential():
    """Plummer sphere truncated at R: inside R its potential is the closed form
    -GM / sqrt(r^2 + a^2) plus the constant G M a^2 / (R^2 + a^2)^(3/2) of the
    removed envelope (integrate 4 pi r rho from r to R: the envelope term is
    (GM/a)[(1 + r^2/a^2)^(-3/2) - (1 + R^2/a^2)^(-3/2)]).  The direct sum leaves
    out each target's own cell (no self term); its continuum share, the potential
    of a homogeneous cube at its centre, is added back so that what remains is
    the second-order error of point masses at the cell centres."""
    a, M, R = 0.1, 1.0, 0.45
    errs = []
    for nbase in (2, 4, 8):
        g = plummer_sphere(a=a, mass=M, r_trunc=R, nbase=nbase)
        t = OracleTree(g)
        x, y, z, m = t.cells()
        c = np.array(g.meta["centre"])
        r = np.sqrt((x - c[0]) ** 2 + (y - c[1]) ** 2 + (z - c[2]) ** 2)
        inside = np.nonzero(r < 0.4)[0]
        tg = inside[_sample_targets(len(inside), 400, seed=nbase)]
        h = g.box_size / (8 * nbase)
        own = np.array([prism_potential(x[i], y[i], z[i], (x[i] - h / 2, y[i] - h / 2, z[i] - h / 2),
                                        (x[i] + h / 2, y[i] + h / 2, z[i] + h / 2), m[i] / h ** 3)
                        for i in tg]).ravel()
        phi = t.direct(tg) + own
        exact = plummer_potential(r[tg], M, a) + M * a * a / (R * R + a * a) ** 1.5
        errs.append(float(np.sqrt(np.mean(((phi - exact) / exact) ** 2))))
    # smooth density sampled at cell centres: second order in h (two halvings: 16x)
    assert errs[0] > errs[1] > errs[2]
    assert errs[0] / errs[2] > 10.0
    assert errs[2] < 5e-4
