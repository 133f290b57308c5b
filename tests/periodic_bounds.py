"""Derived error bounds of the periodic walk and sum against the oracle's
exact Ewald sums (shared by the periodic GPU tests).  Box side 1, table of
N_TABLE^3 points on [0, 1/2]^3 (spacing sp = 1/64).

* Table: D by its third-order expansion, remainder |D^(4)| |delta|^4 / 24,
  the Hessian by its first-order expansion, remainder |D^(4)| |delta|^2 / 2,
  with |D^(4)| <= 24 / (L/2)^5 (the nearest image singularity is at least L/2
  away; the smooth rest of D adds far less) and |delta| <= sqrt(3) sp / 2.
* Storage: the walks read compact rows with H L^3 and T L^4 at half the
  walk's precision (fp32 in the fp64 rows, fp16 in the fp32 rows; unit
  roundoff eps).  With |u_a| <= sp / (2L) per axis and Hs, Ts the table's
  largest |H| L^3 and |T| L^4, the rounding changes D by at most
  eps (Hs (3u)^2 / 2 + Ts (3u)^3 / 6) / L per unit mass and the Hessian by at
  most eps (Hs + 3u Ts) / L^3 per unit of sum_ab |Q_ab| / 6.
* Group-centre cubic (fp32 walks, groups of small cells): the same
  expansions reach |delta| <= sqrt(3) sp / 2 + |u|max, u the offset of a cell
  from the cubic's centre: that of its 4x4x4 octant (|u_a| <= 1.5 h per axis)
  or, for somewhat larger cells, that of its bottom node (|u_a| <= h / 2).  The
  bounds above are taken at that reach (local_reach) and the storage terms
  with |u_a| <= sp / (2L) + u_axis / L.
"""
import numpy as np

N_TABLE = 33
D4 = 24.0 * 2.0 ** 5
DELTA = np.sqrt(3.0) / 64 / 2
TABLE_ERR = D4 * DELTA ** 4 / 24   # per unit mass, about 1e-6
HESS_ERR = D4 * DELTA ** 2 / 2     # per unit of sum_ab |Q_ab| / 6, about 0.07
EPS_FP32_ROWS = 2.0 ** -11         # fp16 storage in the fp32 walks' rows
EPS_FP64_ROWS = 2.0 ** -24         # fp32 storage in the fp64 rows


AXIS_OCTANT, AXIS_NODE = 1.5, 0.5  # largest per-axis offset of a cell from the cubic's centre, in cell sides


def storage_terms(table_values, L, eps, u_axis=0.0):
    """(per unit mass, per unit of sum |Q| / 6) changes from the rows' storage;
    table_values: the fp64 export [n, n, n, 20]; u_axis: the largest per-axis
    offset of a cell from the centre of its group-centre cubic (0: pair
    lookups)."""
    v = table_values.reshape(-1, 20)
    Hs = np.max(np.abs(v[:, 4:10])) * L ** 3
    Ts = np.max(np.abs(v[:, 10:20])) * L ** 4
    u3 = 3 * ((0.5 * L / (N_TABLE - 1)) / (2 * L) + u_axis / L)
    return eps * (0.5 * Hs * u3 ** 2 + Ts * u3 ** 3 / 6) / L, eps * (Hs + u3 * Ts) / L ** 3


def local_reach(h, L, axis=AXIS_OCTANT):
    """|delta| / L the group-centre cubic reaches for cells of side h whose per-axis offset from its centre is at
    most axis * h."""
    return DELTA + np.sqrt(3.0) * axis * h / L


def local_hmax(budget, L, axis=AXIS_OCTANT):
    """Largest cell side taking a cubic with that spread at an error budget (per unit mass, units of 1/L):
    D4 reach^4 / 24 <= budget."""
    u = (budget * 24.0 / D4) ** 0.25 - DELTA
    return max(u, 0.0) * L / (np.sqrt(3.0) * axis)


def local_axis(h, budget, L):
    """Per-axis spread (in cell sides) of the cubic a group of cells of side h takes in an fp32 periodic walk:
    AXIS_OCTANT, AXIS_NODE, or 0 (every pair looked up)."""
    if h <= local_hmax(budget, L, AXIS_OCTANT):
        return AXIS_OCTANT
    if h <= local_hmax(budget, L, AXIS_NODE):
        return AXIS_NODE
    return 0.0


def walk_tolerance(masses_sum, qsum, L, storage, fp32, delta=DELTA):
    """Per-group bound: table (D and, weighted by the group's far-node sum |Q| / 6, the Hessian, both at the
    expansion's reach delta), storage, and in fp32 the rounding of O(1) terms (relative 1e-6 of sum m / d over the
    box, about 3 sum m / L) that cancel to the small periodic potential."""
    ds, hs = storage
    tol = D4 * delta ** 4 / 24 * masses_sum / L + D4 * delta ** 2 / 2 * qsum / L ** 3 + ds * masses_sum + hs * qsum
    if fp32:
        tol = tol + 3e-6 * 3 * masses_sum / L
    return tol


def measured_lookup_errors(table_values, L, n_points=4000, seed=0):
    """Largest errors of the table lookup itself, measured: at random points of
    the octant [0, L/2]^3, D by its third-order Taylor expansion about the
    nearest table point and the Hessian by its first-order one (the lookup the
    walks make, evaluated in fp64 from the exported fp64 table), against the
    oracle's Ewald sums.  Returns (D error per unit mass, largest Hessian-entry
    error), the measured counterparts of TABLE_ERR / L and HESS_ERR / L^3."""
    from oracle.oracle import ewald_hessian
    n = table_values.shape[0]
    v = table_values.reshape(-1, 20)
    sp = 0.5 * L / (n - 1)
    rng = np.random.default_rng(seed)
    u = rng.uniform(0.0, 0.5 * L, (n_points, 3))
    idx = np.clip(np.rint(u / sp).astype(np.int64), 0, n - 1)
    d = u - idx * sp
    row = v[(idx[:, 2] * n + idx[:, 1]) * n + idx[:, 0]]
    x, y, z = d[:, 0], d[:, 1], d[:, 2]
    D0, g, H, T = row[:, 0], row[:, 1:4], row[:, 4:10], row[:, 10:20]
    Txxx, Tyyy, Tzzz, Txxy, Txxz, Txyy, Tyyz, Txzz, Tyzz, Txyz = T.T
    quad = H[:, 0] * x * x + H[:, 1] * y * y + H[:, 2] * z * z + 2 * (H[:, 3] * x * y + H[:, 4] * x * z + H[:, 5] * y * z)
    cube = (Txxx * x ** 3 + Tyyy * y ** 3 + Tzzz * z ** 3 + 3 * (Txxy * x * x * y + Txxz * x * x * z + Txyy * x * y * y
            + Tyyz * y * y * z + Txzz * x * z * z + Tyzz * y * z * z) + 6 * Txyz * x * y * z)
    D = D0 + (g * d).sum(1) + quad / 2 + cube / 6
    Hl = np.stack([H[:, 0] + Txxx * x + Txxy * y + Txxz * z, H[:, 1] + Txyy * x + Tyyy * y + Tyyz * z,
                   H[:, 2] + Txzz * x + Tyzz * y + Tzzz * z, H[:, 3] + Txxy * x + Txyy * y + Txyz * z,
                   H[:, 4] + Txxz * x + Txyz * y + Txzz * z, H[:, 5] + Txyz * x + Tyyz * y + Tyzz * z], 1)
    De, _, He = ewald_hessian(u, L)
    return float(np.max(np.abs(D - De))), float(np.max(np.abs(Hl - He)))
