"""Closed-form potentials used to pin the oracle (test infrastructure only).

Sign convention throughout: phi < 0 (attractive), phi -> -G M / r far away.

* uniform sphere (textbook): -G M / r outside, -2 pi G rho (R^2 - r^2/3) inside;
* MacLaurin spheroid, section "Accuracy with the MacLaurin Sphere": the paper
  prints Chandrasekhar's positive potential V with two slips.  Read here as

    interior  phi = -pi G rho [2 A1 a1^2 - A1 (x^2+y^2) + A3 (a3^2 - z^2)]
    exterior  phi = -(2 a3 / e^2) pi G rho [a1 e atan h
                     - (1 / (2 a1 e)) ((x^2+y^2)(atan h - h/(1+h^2)) + 2 z^2 (h - atan h))]

  with h = a1 e / sqrt(a3^2 + lambda) and lambda the positive root of
  x^2/(a1^2+l) + y^2/(a1^2+l) + z^2/(a3^2+l) = 1.  (The printed interior bracket
  has -A3(a3^2 - z^2) and the printed exterior bracket lacks the 1/(a1 e)
  factor; both readings are pinned against the general ellipsoid integral in
  the tests.)
* homogeneous ellipsoid, general integral form (independent route):
    phi = -pi G rho a1 a2 a3 int_lam^inf (1 - sum x_i^2/(a_i^2+u)) du / Delta(u),
    Delta = sqrt((a1^2+u)(a2^2+u)(a3^2+u)), lam = 0 inside;
* homogeneous rectangular prism (Nagy 1966 / Waldvogel 1979 closed form);
* Plummer sphere: -G M / sqrt(r^2 + a^2).
"""
from __future__ import annotations

import math

import numpy as np


def sphere_potential(r, R, rho, G=1.0):
    r = np.asarray(r, dtype=np.float64)
    M = 4.0 / 3.0 * math.pi * R ** 3 * rho
    out = np.where(r >= R, -G * M / np.maximum(r, 1e-300), -2.0 * math.pi * G * rho * (R * R - r * r / 3.0))
    return out


def maclaurin_A(e):
    s = math.sqrt(1.0 - e * e)
    A1 = s / e ** 3 * math.asin(e) - (1.0 - e * e) / (e * e)
    A3 = 2.0 / (e * e) - 2.0 * s / e ** 3 * math.asin(e)
    return A1, A3


def maclaurin_potential(x, y, z, e, a1, rho, G=1.0):
    """Potential of a homogeneous oblate spheroid (axis z) centred at the origin."""
    x, y, z = (np.asarray(v, dtype=np.float64) for v in (x, y, z))
    a3 = a1 * math.sqrt(1.0 - e * e)
    A1, A3 = maclaurin_A(e)
    R2 = x * x + y * y
    z2 = z * z
    inside = R2 / (a1 * a1) + z2 / (a3 * a3) <= 1.0
    phi_in = -math.pi * G * rho * (2.0 * A1 * a1 * a1 - A1 * R2 + A3 * (a3 * a3 - z2))
    # lambda: positive root of R2/(a1^2+l) + z2/(a3^2+l) = 1  ->  quadratic in l
    b = a1 * a1 + a3 * a3 - R2 - z2
    c = a1 * a1 * a3 * a3 - R2 * a3 * a3 - z2 * a1 * a1
    lam = 0.5 * (-b + np.sqrt(np.maximum(b * b - 4.0 * c, 0.0)))
    lam = np.maximum(lam, 0.0)
    h = a1 * e / np.sqrt(a3 * a3 + lam)
    ath = np.arctan(h)
    phi_out = -(2.0 * a3 / (e * e)) * math.pi * G * rho * (
        a1 * e * ath - (1.0 / (2.0 * a1 * e)) * (R2 * (ath - h / (1.0 + h * h)) + 2.0 * z2 * (h - ath)))
    return np.where(inside, phi_in, phi_out)


def ellipsoid_potential_integral(x, y, z, axes, rho, G=1.0):
    """General homogeneous-ellipsoid potential by adaptive quadrature (one point)."""
    from scipy import integrate, optimize

    a = np.asarray(axes, dtype=np.float64)
    p = np.array([x, y, z], dtype=np.float64)
    F = float(np.sum(p * p / (a * a)))
    if F <= 1.0:
        lam = 0.0
    else:
        f = lambda l: float(np.sum(p * p / (a * a + l))) - 1.0  # noqa: E731
        hi = 1.0
        while f(hi) > 0:
            hi *= 2.0
        lam = optimize.brentq(f, 0.0, hi, xtol=1e-300, rtol=1e-15, maxiter=500)

    def integrand(t):
        # substitution u = lam + t/(1-t) maps [0,1) to [lam, inf)
        u = lam + t / (1.0 - t)
        du = 1.0 / (1.0 - t) ** 2
        D = math.sqrt((a[0] ** 2 + u) * (a[1] ** 2 + u) * (a[2] ** 2 + u))
        return (1.0 - float(np.sum(p * p / (a * a + u)))) / D * du

    val, _ = integrate.quad(integrand, 0.0, 1.0, epsabs=0.0, epsrel=1e-13, limit=400)
    return -math.pi * G * rho * a[0] * a[1] * a[2] * val


def prism_potential(x, y, z, lo, hi, rho, G=1.0):
    """Potential of a homogeneous box [lo, hi] at points (x, y, z) (Nagy/Waldvogel)."""
    x, y, z = (np.asarray(v, dtype=np.float64) for v in (x, y, z))
    total = np.zeros(np.broadcast(x, y, z).shape)
    for i, X in enumerate((lo[0] - x, hi[0] - x)):
        for j, Y in enumerate((lo[1] - y, hi[1] - y)):
            for k, Z in enumerate((lo[2] - z, hi[2] - z)):
                s = (-1.0) ** (i + j + k + 1)  # + at (hi,hi,hi)
                r = np.sqrt(X * X + Y * Y + Z * Z)
                with np.errstate(divide="ignore", invalid="ignore"):
                    t = (X * Y * _safe_log(Z + r) + Y * Z * _safe_log(X + r) + Z * X * _safe_log(Y + r)
                         - 0.5 * X * X * _safe_atan(Y * Z, X * r)
                         - 0.5 * Y * Y * _safe_atan(Z * X, Y * r)
                         - 0.5 * Z * Z * _safe_atan(X * Y, Z * r))
                total = total + s * t
    return -G * rho * total


def _safe_log(v):
    return np.where(v > 0, np.log(np.where(v > 0, v, 1.0)), 0.0)


def _safe_atan(num, den):
    return np.where(den != 0, np.arctan(num / np.where(den != 0, den, 1.0)), 0.0)


def plummer_potential(r, M, a, G=1.0):
    r = np.asarray(r, dtype=np.float64)
    return -G * M / np.sqrt(r * r + a * a)
