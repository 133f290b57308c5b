"""Synthetic block-structured AMR meshes with FP64 cell densities.

Mesh model (PARAMESH-like, as the paper's host code receives it from FLASH4):

* the box ``[box_lo, box_lo + box_size]^3`` is tiled by ``nbase^3`` level-0 blocks
  (``nbase`` a power of two);
* every block holds ``8^3`` cells; a refined block is split into 8 children of
  half the edge, numbered by octant ``o = ox + 2*oy + 4*oz``;
* only leaf blocks carry data.  Densities are stored per leaf, in the order the
  leaves appear in the block list, as ``rho[leaf][z][y][x]`` (x fastest).
* refinement is 2:1 balanced across faces, edges and corners.

Bodies with a sharp edge (sphere, spheroid) are voxelised by volume fraction:
a cell wholly inside or outside the convex body is classified exactly, the
rest by 8^3 sub-sampling, and ``rho = rho_out + (rho_in - rho_out) * f``.

Everything here is deterministic given its arguments (seeded where random).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

NB = 8  # cells per block edge


@dataclass
class AMRGrid:
    name: str
    box_lo: np.ndarray      # (3,) float64
    box_size: float
    nbase: int              # level-0 blocks per dimension
    level: np.ndarray       # int32 [nblk]
    lo: np.ndarray          # float64 [nblk, 3] lower corner
    parent: np.ndarray      # int32 [nblk], -1 for level-0 blocks
    child: np.ndarray       # int32 [nblk, 8], -1 where absent (leaves)
    is_leaf: np.ndarray     # uint8 [nblk]
    rho: np.ndarray         # float64 [nleaf, 8, 8, 8], [z][y][x]
    meta: dict = field(default_factory=dict)

    @property
    def nblocks(self) -> int:
        return int(self.level.shape[0])

    @property
    def leaf_blocks(self) -> np.ndarray:
        return np.nonzero(self.is_leaf)[0].astype(np.int32)

    @property
    def nleaf(self) -> int:
        return int(self.is_leaf.sum())

    @property
    def ncells(self) -> int:
        return self.nleaf * NB ** 3

    def block_edge(self, level) -> np.ndarray:
        return self.box_size / (self.nbase * np.power(2.0, np.asarray(level)))

    def cell_centres(self) -> np.ndarray:
        """Cell-centre coordinates, shape [nleaf, 8, 8, 8, 3] (x, y, z last)."""
        lb = self.leaf_blocks
        h = self.block_edge(self.level[lb]) / NB
        off = np.arange(NB) + 0.5
        lo = self.lo[lb]
        x = lo[:, 0, None] + off[None, :] * h[:, None]
        y = lo[:, 1, None] + off[None, :] * h[:, None]
        z = lo[:, 2, None] + off[None, :] * h[:, None]
        out = np.empty((len(lb), NB, NB, NB, 3))
        out[..., 0] = x[:, None, None, :]
        out[..., 1] = y[:, None, :, None]
        out[..., 2] = z[:, :, None, None]
        return out

    def cell_volumes(self) -> np.ndarray:
        """Cell volume per leaf block, shape [nleaf]."""
        h = self.block_edge(self.level[self.leaf_blocks]) / NB
        return h ** 3

    def max_level(self) -> int:
        return int(self.level.max())


# --------------------------------------------------------------------------
# block-tree construction
# --------------------------------------------------------------------------

def _children_keys(key):
    L, i, j, k = key
    return [(L + 1, 2 * i + (o & 1), 2 * j + ((o >> 1) & 1), 2 * k + ((o >> 2) & 1)) for o in range(8)]


def _balance(leaves: set, nbase: int) -> set:
    """Refine leaves until no two touching leaves differ by more than one level."""
    leaves = set(leaves)
    offs = [(a, b, c) for a in (-1, 0, 1) for b in (-1, 0, 1) for c in (-1, 0, 1) if (a, b, c) != (0, 0, 0)]
    while True:
        to_refine = set()
        for (L, i, j, k) in leaves:
            if L < 2:
                continue
            n = nbase << L
            for a, b, c in offs:
                ii, jj, kk = i + a, j + b, k + c
                if not (0 <= ii < n and 0 <= jj < n and 0 <= kk < n):
                    continue
                # find the leaf that contains the neighbour cell-block region
                for Lc in range(L - 2, -1, -1):
                    s = L - Lc
                    cand = (Lc, ii >> s, jj >> s, kk >> s)
                    if cand in leaves:
                        to_refine.add(cand)
                        break
        if not to_refine:
            return leaves
        for key in to_refine:
            leaves.discard(key)
            leaves.update(_children_keys(key))


def build_grid(name, nbase, refine_fn, max_level, density_fn, box_lo=(0.0, 0.0, 0.0), box_size=1.0,
               meta=None) -> AMRGrid:
    """Build a balanced AMR grid.

    ``refine_fn(L, lo, edge) -> bool`` decides whether a leaf block at level ``L``
    with lower corner ``lo`` (3,) and edge ``edge`` is split (only while
    ``L < max_level``).  ``density_fn(lo[nleaf,3], h[nleaf]) -> rho[nleaf,8,8,8]``
    fills the leaves.
    """
    assert nbase >= 1 and (nbase & (nbase - 1)) == 0, "nbase must be a power of two"
    box_lo = np.asarray(box_lo, dtype=np.float64)
    base_edge = box_size / nbase

    def lo_of(key):
        L, i, j, k = key
        e = base_edge / (1 << L)
        return box_lo + np.array([i, j, k], dtype=np.float64) * e, e

    leaves = {(0, i, j, k) for i in range(nbase) for j in range(nbase) for k in range(nbase)}
    frontier = list(leaves)
    while frontier:
        nxt = []
        for key in frontier:
            if key[0] >= max_level:
                continue
            lo, e = lo_of(key)
            if refine_fn(key[0], lo, e):
                leaves.discard(key)
                ch = _children_keys(key)
                leaves.update(ch)
                nxt.extend(ch)
        frontier = nxt
    leaves = _balance(leaves, nbase)

    # all blocks = leaves + their ancestors
    blocks = set(leaves)
    for (L, i, j, k) in list(leaves):
        while L > 0:
            L, i, j, k = L - 1, i >> 1, j >> 1, k >> 1
            if (L, i, j, k) in blocks:
                break
            blocks.add((L, i, j, k))
    order = sorted(blocks, key=lambda t: (t[0], t[3], t[2], t[1]))
    index = {key: n for n, key in enumerate(order)}
    nblk = len(order)
    level = np.empty(nblk, np.int32)
    lo = np.empty((nblk, 3), np.float64)
    parent = np.full(nblk, -1, np.int32)
    child = np.full((nblk, 8), -1, np.int32)
    is_leaf = np.zeros(nblk, np.uint8)
    for n, key in enumerate(order):
        level[n] = key[0]
        lo[n], _ = lo_of(key)
        if key in leaves:
            is_leaf[n] = 1
        else:
            for o, ck in enumerate(_children_keys(key)):
                c = index[ck]
                child[n, o] = c
                parent[c] = n
    lb = np.nonzero(is_leaf)[0]
    h = base_edge / np.power(2.0, level[lb]) / NB
    rho = np.ascontiguousarray(density_fn(lo[lb], h), dtype=np.float64)
    assert rho.shape == (len(lb), NB, NB, NB)
    return AMRGrid(name=name, box_lo=box_lo, box_size=float(box_size), nbase=nbase, level=level, lo=lo,
                   parent=parent, child=child, is_leaf=is_leaf, rho=rho, meta=dict(meta or {}))


# --------------------------------------------------------------------------
# voxelisation of a convex, axis-aligned ellipsoid (sphere as special case)
# --------------------------------------------------------------------------

def _interval_min_sq(a, b):
    """min of x^2 over [a, b] (elementwise)."""
    return np.where((a <= 0) & (b >= 0), 0.0, np.minimum(a * a, b * b))


def _interval_max_sq(a, b):
    return np.maximum(a * a, b * b)


def ellipsoid_fraction(lo, h, centre, axes, sub=8):
    """Volume fraction of cells inside ((x-c)/a)^2 + ... <= 1.

    ``lo`` [nleaf,3] block corners, ``h`` [nleaf] cell sizes.  Returns [nleaf,8,8,8].
    Cells entirely inside (max of F over the cell <= 0, F convex so attained at a
    corner) get 1, cells entirely outside (separable min of F > 0) get 0, the
    rest are sub-sampled on a ``sub^3`` lattice of sub-cell centres.
    """
    centre = np.asarray(centre, np.float64)
    axes = np.asarray(axes, np.float64)
    n = lo.shape[0]
    idx = np.arange(NB, dtype=np.float64)
    out = np.zeros((n, NB, NB, NB))
    # per-axis cell bounds relative to the centre, scaled by the semi-axis
    bounds = []
    for d in range(3):
        a = (lo[:, d, None] + idx[None, :] * h[:, None] - centre[d]) / axes[d]
        b = (lo[:, d, None] + (idx[None, :] + 1.0) * h[:, None] - centre[d]) / axes[d]
        bounds.append((a, b))
    (ax, bx), (ay, by), (az, bz) = bounds
    fmin = (_interval_min_sq(az, bz)[:, :, None, None] + _interval_min_sq(ay, by)[:, None, :, None]
            + _interval_min_sq(ax, bx)[:, None, None, :]) - 1.0
    fmax = (_interval_max_sq(az, bz)[:, :, None, None] + _interval_max_sq(ay, by)[:, None, :, None]
            + _interval_max_sq(ax, bx)[:, None, None, :]) - 1.0
    out[fmax <= 0.0] = 1.0
    mixed = np.nonzero((fmin <= 0.0) & (fmax > 0.0))
    if mixed[0].size:
        b_, z_, y_, x_ = mixed
        s = (np.arange(sub) + 0.5) / sub
        hh = h[b_]
        px = (lo[b_, 0] + x_ * hh)[:, None] + s[None, :] * hh[:, None]
        py = (lo[b_, 1] + y_ * hh)[:, None] + s[None, :] * hh[:, None]
        pz = (lo[b_, 2] + z_ * hh)[:, None] + s[None, :] * hh[:, None]
        fx = ((px - centre[0]) / axes[0]) ** 2
        fy = ((py - centre[1]) / axes[1]) ** 2
        fz = ((pz - centre[2]) / axes[2]) ** 2
        inside = (fz[:, :, None, None] + fy[:, None, :, None] + fx[:, None, None, :]) <= 1.0
        out[mixed] = inside.reshape(len(b_), -1).mean(axis=1)
    return out


def _ellipsoid_straddles(lo, e, centre, axes):
    a = (lo - centre) / axes
    b = (lo + e - centre) / axes
    fmin = float(np.sum(_interval_min_sq(a, b))) - 1.0
    fmax = float(np.sum(_interval_max_sq(a, b))) - 1.0
    return fmin <= 0.0 < fmax


# --------------------------------------------------------------------------
# named workloads
# --------------------------------------------------------------------------

def uniform_sphere(radius=0.4, rho_in=1.0, rho_out=1e-3, nbase=4, max_level=0, centre=(0.5, 0.5, 0.5)):
    """Uniform sphere in the unit box; by default 4^3 blocks of 8^3 (32^3 cells).

    With ``max_level > 0`` the blocks straddling the surface are refined.
    """
    c = np.asarray(centre, np.float64)
    ax = np.array([radius] * 3)

    def refine(L, lo, e):
        return _ellipsoid_straddles(lo, e, c, ax)

    def dens(lo, h):
        return rho_out + (rho_in - rho_out) * ellipsoid_fraction(lo, h, c, ax)

    return build_grid("uniform_sphere", nbase, refine, max_level, dens,
                      meta=dict(radius=radius, rho_in=rho_in, rho_out=rho_out, centre=c.tolist()))


def maclaurin_axes(e, a1):
    """Semi-axes (a1, a1, a3) of an oblate spheroid of eccentricity e = sqrt(1 - (a3/a1)^2)."""
    return a1, a1, a1 * math.sqrt(1.0 - e * e)


def maclaurin_spheroid(e=0.9, a1=0.25, rho_in=1.0, rho_out=1e-5, nbase=4, max_level=3,
                       centre=(0.5, 0.5, 0.5)):
    """Homogeneous oblate (MacLaurin) spheroid, symmetry axis z, refined at its surface."""
    c = np.asarray(centre, np.float64)
    ax = np.array(maclaurin_axes(e, a1))

    def refine(L, lo, edge):
        return _ellipsoid_straddles(lo, edge, c, ax)

    def dens(lo, h):
        return rho_out + (rho_in - rho_out) * ellipsoid_fraction(lo, h, c, ax)

    return build_grid("maclaurin_spheroid", nbase, refine, max_level, dens,
                      meta=dict(e=e, a1=a1, a3=float(ax[2]), rho_in=rho_in, rho_out=rho_out, centre=c.tolist()))


def cloud_core(r0=0.02, rho0=1.0, r_trunc=0.5, contrast_out=1e-4, sigma=0.1, seed=1509, nbase=4,
               max_level=7, jeans_cs=None, cells_per_jeans=4.0, centre=(0.5, 0.5, 0.5)):
    """Centrally condensed core rho0 / (1 + (r/r0)^2), truncated at r_trunc, lognormal noise.

    Blocks are refined while the Jeans length sqrt(pi c_s^2 / (G rho_max)) of the
    block's densest point is shorter than ``cells_per_jeans`` cells (G = 1).  If
    ``jeans_cs`` is None it is the largest sound speed (bisection on log c_s)
    for which that criterion still refines down to ``max_level``; with the
    defaults this gives 24256 leaf blocks (12.4M cells) over 8 levels.
    """
    c = np.asarray(centre, np.float64)

    def rho_profile_max(lo, e):
        # densest point of the block: the point nearest the centre
        q = np.clip(c, lo, lo + e)
        r = float(np.linalg.norm(q - c))
        return rho0 / (1.0 + (r / r0) ** 2) if r <= r_trunc else rho0 * contrast_out

    def make_refine(cs):
        def refine(L, lo, e):
            h = e / NB
            rmax = rho_profile_max(lo, e)
            lam = math.sqrt(math.pi * cs * cs / rmax)
            return lam < cells_per_jeans * h
        return refine

    def reaches_max_level(cs):
        # refinement without balance is enough to know the deepest level
        frontier = [(0, np.array([i, j, k], float)) for i in range(nbase) for j in range(nbase)
                    for k in range(nbase)]
        ref = make_refine(cs)
        while frontier:
            nxt = []
            for L, ijk in frontier:
                e = 1.0 / (nbase << L)
                if ref(L, ijk * e, e):
                    if L + 1 == max_level:
                        return True
                    for o in range(8):
                        nxt.append((L + 1, 2 * ijk + np.array([o & 1, (o >> 1) & 1, (o >> 2) & 1], float)))
            frontier = nxt
        return False

    if jeans_cs is None:
        # the largest sound speed whose Jeans criterion still reaches max_level
        lo_cs, hi_cs = -8.0, 2.0  # log10 bracket: refines to max_level at lo, not at hi
        for _ in range(40):
            mid = 0.5 * (lo_cs + hi_cs)
            if reaches_max_level(10.0 ** mid):
                lo_cs = mid
            else:
                hi_cs = mid
        jeans_cs = 10.0 ** lo_cs

    rng = np.random.default_rng(seed)

    def dens(lo, h):
        off = np.arange(NB) + 0.5
        x = lo[:, 0, None] + off[None, :] * h[:, None]
        y = lo[:, 1, None] + off[None, :] * h[:, None]
        z = lo[:, 2, None] + off[None, :] * h[:, None]
        r2 = ((z[:, :, None, None] - c[2]) ** 2 + (y[:, None, :, None] - c[1]) ** 2
              + (x[:, None, None, :] - c[0]) ** 2)
        r = np.sqrt(r2)
        base = np.where(r <= r_trunc, rho0 / (1.0 + r2 / (r0 * r0)), rho0 * contrast_out)
        z_ = rng.standard_normal(base.shape)
        return base * np.exp(sigma * z_ - 0.5 * sigma * sigma)

    return build_grid("cloud_core", nbase, make_refine(jeans_cs), max_level, dens,
                      meta=dict(r0=r0, rho0=rho0, r_trunc=r_trunc, contrast_out=contrast_out, sigma=sigma,
                                seed=seed, jeans_cs=jeans_cs, cells_per_jeans=cells_per_jeans))


def plummer_mix(seed, n_target_blocks=None, nbase=4, max_level=None):
    """Seeded mix of 1-4 Plummer spheres rho = (3M / 4 pi a^3)(1 + r^2/a^2)^(-5/2).

    Scale a log-uniform in [0.02, 0.1], mass ratios uniform in [0.1, 1], centres
    uniform in [0.3, 0.7]^3, max level uniform in {3..6} unless given; blocks
    are refined in order of decreasing peak density until the leaf-block target
    (log-uniform in [100, 8000] unless given) would be exceeded.  The random
    draws do not depend on the arguments given.
    """
    rng = np.random.default_rng(seed)
    k = int(rng.integers(1, 5))
    a = np.exp(rng.uniform(math.log(0.02), math.log(0.1), size=k))
    mass = rng.uniform(0.1, 1.0, size=k)
    ctr = rng.uniform(0.3, 0.7, size=(k, 3))
    drawn_level = int(rng.integers(3, 7))
    max_level = drawn_level if max_level is None else int(max_level)
    if n_target_blocks is None:
        n_target_blocks = int(round(math.exp(rng.uniform(math.log(100), math.log(8000)))))

    def rho_at(p):
        out = np.zeros(p.shape[:-1])
        for s in range(k):
            r2 = np.sum((p - ctr[s]) ** 2, axis=-1)
            out += 3.0 * mass[s] / (4.0 * math.pi * a[s] ** 3) * (1.0 + r2 / a[s] ** 2) ** -2.5
        return out

    def peak(lo, e):
        q = np.clip(ctr, lo, lo + e)
        best = 0.0
        for s in range(k):
            # density of component s at its nearest point plus the others there
            best = max(best, float(rho_at(q[s][None, :])[0]))
        return best

    # greedy refinement by peak density (a priority order) up to the block target
    leaves = {(0, i, j, k_) for i in range(nbase) for j in range(nbase) for k_ in range(nbase)}
    import heapq
    heap = []

    def push(key):
        L, i, j, k_ = key
        e = 1.0 / (nbase << L)
        lo = np.array([i, j, k_], float) * e
        heapq.heappush(heap, (-peak(lo, e) * e ** 3 * (1 << (2 * L)), key))

    for key in leaves:
        push(key)
    while heap and len(leaves) + 7 <= n_target_blocks:
        _, key = heapq.heappop(heap)
        if key[0] >= max_level or key not in leaves:
            continue
        leaves.discard(key)
        for ck in _children_keys(key):
            leaves.add(ck)
            push(ck)
    chosen = set(leaves)

    # refine exactly the ancestors of the chosen leaves
    anc = set()
    for (L, i, j, k_) in chosen:
        while L > 0:
            L, i, j, k_ = L - 1, i >> 1, j >> 1, k_ >> 1
            anc.add((L, i, j, k_))

    def refine_anc(L, lo, e):
        i, j, k_ = (np.round(lo * (nbase << L))).astype(int)
        return (L, int(i), int(j), int(k_)) in anc

    def dens(lo, h):
        off = np.arange(NB) + 0.5
        x = lo[:, 0, None] + off[None, :] * h[:, None]
        y = lo[:, 1, None] + off[None, :] * h[:, None]
        z = lo[:, 2, None] + off[None, :] * h[:, None]
        p = np.empty((lo.shape[0], NB, NB, NB, 3))
        p[..., 0] = x[:, None, None, :]
        p[..., 1] = y[:, None, :, None]
        p[..., 2] = z[:, :, None, None]
        return rho_at(p)

    return build_grid("plummer_mix", nbase, refine_anc, max_level, dens,
                      meta=dict(seed=seed, k=k, a=a.tolist(), mass=mass.tolist(), centres=ctr.tolist(),
                                max_level=max_level, n_target_blocks=n_target_blocks))


def random_amr(seed, nbase=2, max_level=2, p_refine=0.3, sigma=1.0, zero_fraction=0.0):
    """Small random AMR grid with lognormal densities (for parity tests).

    Each block is refined with probability ``p_refine`` (seeded), then balanced.
    A fraction ``zero_fraction`` of leaf blocks gets zero density (exercises
    zero-mass nodes).
    """
    rng = np.random.default_rng(seed)
    decisions = {}

    def refine(L, lo, e):
        key = (L, tuple(np.round(lo / e).astype(int)))
        if key not in decisions:
            decisions[key] = bool(rng.random() < p_refine)
        return decisions[key]

    def dens(lo, h):
        r = np.exp(sigma * rng.standard_normal((lo.shape[0], NB, NB, NB)))
        if zero_fraction > 0:
            z = rng.random(lo.shape[0]) < zero_fraction
            r[z] = 0.0
        return r

    return build_grid("random_amr", nbase, refine, max_level, dens,
                      meta=dict(seed=seed, p_refine=p_refine, sigma=sigma, zero_fraction=zero_fraction))


def single_block(seed=0, sigma=0.5):
    """One 8^3 block covering the unit box (the smallest grid)."""
    rng = np.random.default_rng(seed)

    def dens(lo, h):
        return np.exp(sigma * rng.standard_normal((lo.shape[0], NB, NB, NB)))

    return build_grid("single_block", 1, lambda *a: False, 0, dens, meta=dict(seed=seed))


def plummer_sphere(a=0.1, mass=1.0, r_trunc=0.45, nbase=4, max_level=0, centre=(0.5, 0.5, 0.5)):
    """One Plummer sphere rho = (3M / 4 pi a^3)(1 + r^2/a^2)^(-5/2), zero beyond r_trunc.

    Densities are sampled at the cell centres and weighted by the cell's
    volume fraction inside r_trunc.  With ``max_level > 0`` the
    blocks within 2a of the centre are refined.
    """
    c = np.asarray(centre, np.float64)

    def refine(L, lo, e):
        q = np.clip(c, lo, lo + e)
        return float(np.sqrt(((q - c) ** 2).sum())) < 2 * a

    def dens(lo, h):
        off = np.arange(NB) + 0.5
        x = lo[:, 0, None] + off[None, :] * h[:, None] - c[0]
        y = lo[:, 1, None] + off[None, :] * h[:, None] - c[1]
        z = lo[:, 2, None] + off[None, :] * h[:, None] - c[2]
        r2 = x[:, None, None, :] ** 2 + y[:, None, :, None] ** 2 + z[:, :, None, None] ** 2
        rho = 3.0 * mass / (4.0 * math.pi * a ** 3) * (1.0 + r2 / a ** 2) ** -2.5
        return rho * ellipsoid_fraction(lo, h, c, np.array([r_trunc] * 3))

    return build_grid("plummer_sphere", nbase, refine, max_level, dens,
                      meta=dict(a=a, mass=mass, r_trunc=r_trunc, centre=c.tolist()))
