"""ctypes front-end of the plain-C FP64 oracle (``bh_oracle.c``).

Test infrastructure only: nothing in the product package imports this module.
Each method names the definition it follows (see the header of bh_oracle.c):
O1 cells, O2 direct sum, O3 node moments, O4-O6 group walk, O7 potential sum,
O8 accelerations, O9 the periodic Green's function, O10 the periodic walk and sum.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "bh_oracle.c")
_LIB = os.path.join(_HERE, "libbh_oracle.so")
_lock = threading.Lock()
_lib = None

# Portable flags: the built library may run on another x86-64 host.  FP
# contraction is off so that d^2 = dx*dx + dy*dy + dz*dz rounds as written.
CFLAGS = ["-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared"]


def oracle_library_path() -> str:
    return _LIB


def build_oracle(force: bool = True) -> str:
    """Compile bh_oracle.c with gcc into oracle/libbh_oracle.so."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", *CFLAGS, _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build_oracle(force=True)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        i64 = ctypes.c_int64
        lib.ot_create.restype = P
        lib.ot_create.argtypes = [ctypes.c_int, P, P, P, P, P, P, ctypes.c_double, ctypes.c_int]
        lib.ot_destroy.argtypes = [P]
        lib.ot_num_nodes.restype = ctypes.c_int
        lib.ot_num_nodes.argtypes = [P]
        lib.ot_num_cells.restype = i64
        lib.ot_num_cells.argtypes = [P]
        lib.ot_num_leaves.restype = ctypes.c_int
        lib.ot_num_leaves.argtypes = [P]
        lib.ot_node_info.argtypes = [P, P, P, P, P, P]
        lib.ot_lookup.restype = ctypes.c_int
        lib.ot_lookup.argtypes = [P, ctypes.c_uint64]
        lib.ot_make_key.restype = ctypes.c_uint64
        lib.ot_make_key.argtypes = [ctypes.c_int, i64, i64, i64]
        lib.ot_set_density.argtypes = [P, P]
        lib.ot_moments.argtypes = [P]
        lib.ot_get_moments.argtypes = [P, P, P, P, P]
        lib.ot_walk.restype = i64
        lib.ot_walk.argtypes = [P, ctypes.c_int, P, ctypes.c_double]
        lib.ot_walk_mac.restype = i64
        lib.ot_walk_mac.argtypes = [P, ctypes.c_int, P, ctypes.c_double, ctypes.c_int]
        lib.ot_solve_groups_mac.argtypes = [P, ctypes.c_int, P, P, i64, ctypes.c_double, ctypes.c_double,
                                            ctypes.c_int, ctypes.c_int, P, P]
        lib.ot_walk_sizes.argtypes = [P, P, P]
        lib.ot_walk_export.argtypes = [P, P, P, P, P, P]
        lib.ot_potential.argtypes = [P, ctypes.c_double, ctypes.c_int, P]
        lib.ot_potential_lists.restype = ctypes.c_int
        lib.ot_potential_lists.argtypes = [P, ctypes.c_int, P, P, P, P, ctypes.c_double, ctypes.c_int, P]
        lib.ot_direct.argtypes = [P, P, i64, ctypes.c_double, P]
        lib.ot_set_threads.argtypes = [ctypes.c_int]
        lib.ot_set_tau_lin.argtypes = [P, ctypes.c_double]
        lib.ot_get_threads.restype = ctypes.c_int
        lib.ot_solve_groups.argtypes = [P, ctypes.c_int, P, P, i64, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                        P, P]
        lib.ot_cells.argtypes = [P, P, P, P, P]
        lib.ot_accel.argtypes = [P, ctypes.c_double, ctypes.c_int, P]
        lib.ot_solve_groups_accel.argtypes = [P, ctypes.c_int, P, P, i64, ctypes.c_double, ctypes.c_double,
                                              ctypes.c_int, P, P]
        lib.ot_direct_accel.argtypes = [P, P, i64, ctypes.c_double, P]
        lib.ot_direct_at.argtypes = [P, P, P, i64, ctypes.c_double, P]
        lib.ot_ewald.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_int, ctypes.c_int, P, i64, P, P]
        lib.ot_direct_periodic.argtypes = [P, P, i64, ctypes.c_double, P]
        lib.ot_get_trace.argtypes = [P, P]
        lib.ot_ewald_hessian.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_int, ctypes.c_int, P, i64, P, P,
                                         P]
        lib.ot_solve_groups_periodic.argtypes = [P, ctypes.c_int, P, P, i64, ctypes.c_double, ctypes.c_double, P, P,
                                                 P]
        lib.ot_node_far_periodic.argtypes = [P, ctypes.c_int, P, P]
        _lib = lib
        return lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def set_threads(n):
    """Threads of the oracle's OpenMP regions; returns what the runtime reports it will use."""
    lib = _load()
    lib.ot_set_threads(int(n))
    return int(lib.ot_get_threads())


def get_threads():
    return int(_load().ot_get_threads())


U32 = 2.0 ** -24  # unit roundoff of fp32


def fp32_band_for(B):
    """fp32_band for coordinates of magnitude at most B."""
    return (18.0 * U32, 12.0 * np.sqrt(3.0) * U32 * float(B))


def fp32_band(grid):
    """Marginal band (tau, tau_lin) of an fp32 opening test on `grid`, from the fp32
    rounding of its operands: per axis the gap between a cell centre and a node's
    centre of mass is off by at most 3 u B (B the largest coordinate of the box:
    both rounded to fp32, then subtracted), so d^2 moves by at most
    2 sqrt(3) d 3 u B + 3 u d^2; s = l / theta + delta by 3 u s, s^2 by 6 u s^2.
    Near the threshold (d ~ s): |d^2 - s^2| changes by at most 9 u s^2 + 6 sqrt(3) u B s.
    Twice that: tau = 18 u, tau_lin = 12 sqrt(3) u B."""
    lo = np.asarray(grid.box_lo, np.float64)
    return fp32_band_for(np.max(np.abs(np.concatenate([lo, lo + grid.box_size]))))


def make_key(depth, ix, iy, iz):
    """Node identity shared by every implementation: (depth, corner / edge)."""
    return (np.uint64(depth) << np.uint64(57)) | (np.uint64(ix) << np.uint64(38)) | \
        (np.uint64(iy) << np.uint64(19)) | np.uint64(iz)


def split_key(keys):
    k = np.asarray(keys, dtype=np.uint64)
    m = np.uint64((1 << 19) - 1)
    return ((k >> np.uint64(57)).astype(np.int64), ((k >> np.uint64(38)) & m).astype(np.int64),
            ((k >> np.uint64(19)) & m).astype(np.int64), (k & m).astype(np.int64))


class OracleTree:
    """Octree of an AMR grid as the oracle builds it (own code, own node order)."""

    def __init__(self, grid):
        self.lib = _load()
        self.grid = grid
        self._keep = [np.ascontiguousarray(grid.level, np.int32), np.ascontiguousarray(grid.lo, np.float64),
                      np.ascontiguousarray(grid.parent, np.int32), np.ascontiguousarray(grid.child, np.int32),
                      np.ascontiguousarray(grid.is_leaf, np.uint8), np.ascontiguousarray(grid.box_lo, np.float64)]
        lv, lo, pa, ch, il, bl = self._keep
        self.h = ctypes.c_void_p(self.lib.ot_create(grid.nblocks, _p(lv), _p(lo), _p(pa), _p(ch), _p(il), _p(bl),
                                                    float(grid.box_size), int(grid.nbase)))
        self.nnodes = self.lib.ot_num_nodes(self.h)
        self.ncells = self.lib.ot_num_cells(self.h)
        self.nleaf = self.lib.ot_num_leaves(self.h)
        self._density_set = False
        self._moments_done = False
        self.group_cells = None

    def __del__(self):
        try:
            if getattr(self, "h", None):
                self.lib.ot_destroy(self.h)
                self.h = None
        except Exception:
            pass

    def _band(self, tau):
        """tau: a relative band, or (relative, linear) as fp32_band gives: sets the linear term for the next walk
        and returns the relative one."""
        if isinstance(tau, (tuple, list)):
            rel, lin = float(tau[0]), float(tau[1])
        else:
            rel, lin = float(tau), 0.0
        self.lib.ot_set_tau_lin(self.h, lin)
        return rel

    # -- geometry -----------------------------------------------------------
    def node_info(self):
        n = self.nnodes
        key = np.empty(n, np.uint64)
        depth = np.empty(n, np.int32)
        bottom = np.empty(n, np.int32)
        centre = np.empty((n, 3))
        edge = np.empty(n)
        self.lib.ot_node_info(self.h, _p(key), _p(depth), _p(bottom), _p(centre), _p(edge))
        return dict(key=key, depth=depth, bottom=bottom, centre=centre, edge=edge)

    def cells(self):
        """O1: cell centres and masses in caller order (leaf, z, y, x)."""
        if not self._density_set:
            self.set_density()
        n = self.ncells
        x, y, z, m = (np.empty(n) for _ in range(4))
        self.lib.ot_cells(self.h, _p(x), _p(y), _p(z), _p(m))
        return x, y, z, m

    # -- O1 / O3 --------------------------------------------------------------
    def set_density(self, rho=None):
        rho = np.ascontiguousarray(self.grid.rho if rho is None else rho, np.float64)
        assert rho.size == self.ncells
        self.lib.ot_set_density(self.h, _p(rho))
        self._density_set = True
        self._moments_done = False

    def moments(self):
        """O3: brute-force moments of every node; returns arrays keyed by node key."""
        if not self._density_set:
            self.set_density()
        if not self._moments_done:
            self.lib.ot_moments(self.h)
            self._moments_done = True
        n = self.nnodes
        M = np.empty(n)
        X = np.empty((n, 3))
        Q = np.empty((n, 6))
        d = np.empty(n)
        self.lib.ot_get_moments(self.h, _p(M), _p(X), _p(Q), _p(d))
        S = np.empty(n)
        self.lib.ot_get_trace(self.h, _p(S))
        info = self.node_info()
        info.update(M=M, X=X, Q=Q, delta=d, S=S)
        return info

    # -- O4-O6 -----------------------------------------------------------------
    def n_groups(self, group_cells):
        return self.nleaf * (512 // group_cells)

    def walk(self, group_cells=64, theta=0.5, tau=0.0, mac=0):
        """O5/O6 for every group; ``theta`` is a scalar or one value per group.
        ``mac`` 0: every cell of the group is tested (O5); 1: the group's cube (O5b)."""
        assert 512 % group_cells == 0 and (group_cells & (group_cells - 1)) == 0
        if not self._moments_done:
            self.moments()
        ng = self.n_groups(group_cells)
        th = np.broadcast_to(np.asarray(theta, np.float64), (ng,)).copy()
        self.lib.ot_walk_mac(self.h, int(group_cells), _p(th), self._band(tau), int(mac))
        self.group_cells = group_cells
        tf = ctypes.c_int64()
        tn = ctypes.c_int64()
        self.lib.ot_walk_sizes(self.h, ctypes.byref(tf), ctypes.byref(tn))
        far_off = np.empty(ng + 1, np.int64)
        near_off = np.empty(ng + 1, np.int64)
        far_keys = np.empty(max(tf.value, 1), np.uint64)
        near_keys = np.empty(max(tn.value, 1), np.uint64)
        counts = np.empty((ng, 4), np.int64)
        self.lib.ot_walk_export(self.h, _p(far_off), _p(far_keys), _p(near_off), _p(near_keys), _p(counts))
        return dict(far_off=far_off, far_keys=far_keys[:tf.value], near_off=near_off,
                    near_keys=near_keys[:tn.value], visited=counts[:, 0], n_far=counts[:, 1],
                    n_near=counts[:, 2], marginal=counts[:, 3])

    # -- O7 ----------------------------------------------------------------------
    def potential(self, G=1.0, order=2):
        """O7 with the lists of the last walk; returns phi[nleaf, 8, 8, 8].

        ``order`` 2 = monopole + quadrupole, 0 = monopole only."""
        assert self.group_cells is not None, "walk() first"
        phi = np.empty(self.ncells)
        self.lib.ot_potential(self.h, float(G), int(order), _p(phi))
        return phi.reshape(self.nleaf, 8, 8, 8)

    def potential_lists(self, group_cells, far_off, far_keys, near_off, near_keys, G=1.0, order=2):
        """O7 evaluated on interaction lists given by node key (list replay)."""
        if not self._moments_done:
            self.moments()
        far_off = np.ascontiguousarray(far_off, np.int64)
        near_off = np.ascontiguousarray(near_off, np.int64)
        fk = np.ascontiguousarray(far_keys, np.uint64)
        nk = np.ascontiguousarray(near_keys, np.uint64)
        if fk.size == 0:
            fk = np.zeros(1, np.uint64)
        if nk.size == 0:
            nk = np.zeros(1, np.uint64)
        assert far_off.size == self.n_groups(group_cells) + 1
        phi = np.empty(self.ncells)
        rc = self.lib.ot_potential_lists(self.h, int(group_cells), _p(far_off), _p(fk), _p(near_off), _p(nk),
                                         float(G), int(order), _p(phi))
        if rc != 0:
            raise ValueError("list replay: %s" % ("unknown node key" if rc == -1 else "near entry not a bottom node"))
        return phi.reshape(self.nleaf, 8, 8, 8)

    def solve_groups(self, groups, group_cells=64, theta=0.5, tau=0.0, G=1.0, order=2, mac=0):
        """O5-O7 for selected canonical groups only.  Returns (phi[n, G] in the
        group's Morton order, counts[n, 4] = visited, far, near, marginal)."""
        if not self._moments_done:
            self.moments()
        ng = self.n_groups(group_cells)
        th = np.broadcast_to(np.asarray(theta, np.float64), (ng,)).copy()
        gs = np.ascontiguousarray(groups, np.int64)
        phi = np.empty((gs.size, group_cells))
        counts = np.empty((gs.size, 4), np.int64)
        self.lib.ot_solve_groups_mac(self.h, int(group_cells), _p(th), _p(gs), int(gs.size), self._band(tau), float(G),
                                     int(order), int(mac), _p(counts), _p(phi))
        return phi, counts

    # -- O9 ----------------------------------------------------------------------
    def direct_periodic(self, targets=None, G=1.0):
        """Exact periodic direct sum (nearest image + Ewald smooth part + self images) at canonical cell ids."""
        if not self._density_set:
            self.set_density()
        t = np.arange(self.ncells, dtype=np.int64) if targets is None else np.ascontiguousarray(targets, np.int64)
        phi = np.empty(t.size)
        self.lib.ot_direct_periodic(self.h, _p(t), int(t.size), float(G), _p(phi))
        return phi

    # -- O10 ---------------------------------------------------------------------
    def solve_groups_periodic(self, groups, group_cells=64, theta=0.5, tau=0.0, G=1.0, with_qsum=False):
        """O10 (periodic walk and sum) for selected canonical groups.  Returns
        (phi[n, G] in the group's Morton order, counts[n, 4] = visited, far, near, marginal), and with
        ``with_qsum`` also qsum[n] = sum over far nodes of sum_ab |Q_ab| / 6."""
        if not self._moments_done:
            self.moments()
        ng = self.n_groups(group_cells)
        th = np.broadcast_to(np.asarray(theta, np.float64), (ng,)).copy()
        gs = np.ascontiguousarray(groups, np.int64)
        phi = np.empty((gs.size, group_cells))
        counts = np.empty((gs.size, 4), np.int64)
        qsum = np.empty(gs.size)
        self.lib.ot_solve_groups_periodic(self.h, int(group_cells), _p(th), _p(gs), int(gs.size), self._band(tau),
                                          float(G), _p(counts), _p(phi), _p(qsum))
        return (phi, counts, qsum) if with_qsum else (phi, counts)

    def node_far_periodic(self, node, point):
        """O10 far term of node id ``node`` at ``point`` by part: M (1/|R| + D), R^T Q R / (2 |R|^5),
        Q:H / 6, 2 pi S / (3 L^3)."""
        if not self._moments_done:
            self.moments()
        p = np.ascontiguousarray(point, np.float64).reshape(3)
        out = np.empty(4)
        self.lib.ot_node_far_periodic(self.h, int(node), _p(p), _p(out))
        return out

    # -- O8 ----------------------------------------------------------------------
    def accel(self, G=1.0, order=2):
        """O8 with the lists of the last walk; returns g[nleaf, 8, 8, 8, 3]."""
        assert self.group_cells is not None, "walk() first"
        acc = np.empty((self.ncells, 3))
        self.lib.ot_accel(self.h, float(G), int(order), _p(acc))
        return acc.reshape(self.nleaf, 8, 8, 8, 3)

    def solve_groups_accel(self, groups, group_cells=64, theta=0.5, tau=0.0, G=1.0, order=2):
        """O5, O6, O8 for selected canonical groups.  Returns (g[n, G, 3] in the
        group's Morton order, counts[n, 4] = visited, far, near, marginal)."""
        if not self._moments_done:
            self.moments()
        ng = self.n_groups(group_cells)
        th = np.broadcast_to(np.asarray(theta, np.float64), (ng,)).copy()
        gs = np.ascontiguousarray(groups, np.int64)
        acc = np.empty((gs.size, group_cells, 3))
        counts = np.empty((gs.size, 4), np.int64)
        self.lib.ot_solve_groups_accel(self.h, int(group_cells), _p(th), _p(gs), int(gs.size), self._band(tau), float(G),
                                       int(order), _p(counts), _p(acc))
        return acc, counts

    def direct_accel(self, targets=None, G=1.0):
        """Exact direct-sum acceleration at canonical cell ids (all if None), [n, 3]."""
        if not self._density_set:
            self.set_density()
        t = np.arange(self.ncells, dtype=np.int64) if targets is None else np.ascontiguousarray(targets, np.int64)
        acc = np.empty((t.size, 3))
        self.lib.ot_direct_accel(self.h, _p(t), int(t.size), float(G), _p(acc))
        return acc

    def direct_at(self, points, exclude, G=1.0):
        """Direct-sum potential at arbitrary points [n, 3], leaving out cell exclude[q] (-1: none)."""
        if not self._density_set:
            self.set_density()
        p = np.ascontiguousarray(points, np.float64).reshape(-1, 3)
        ex = np.ascontiguousarray(np.broadcast_to(np.asarray(exclude, np.int64), (p.shape[0],)))
        phi = np.empty(p.shape[0])
        self.lib.ot_direct_at(self.h, _p(p), _p(ex), int(p.shape[0]), float(G), _p(phi))
        return phi

    # -- O2 ----------------------------------------------------------------------
    def direct(self, targets=None, G=1.0):
        """O2 at canonical cell ids ``targets`` (all cells if None)."""
        if not self._density_set:
            self.set_density()
        t = np.arange(self.ncells, dtype=np.int64) if targets is None else np.ascontiguousarray(targets, np.int64)
        phi = np.empty(t.size)
        self.lib.ot_direct(self.h, _p(t), int(t.size), float(G), _p(phi))
        return phi


def ewald(points, L=1.0, alpha=None, nreal=4, nrecip=5):
    """O9: smooth part D = psi - 1/r of the periodic Green's function and its
    gradient at points [n, 3]; returns (D[n], grad[n, 3])."""
    lib = _load()
    p = np.ascontiguousarray(points, np.float64).reshape(-1, 3)
    D = np.empty(p.shape[0])
    g = np.empty((p.shape[0], 3))
    a = 2.0 / L if alpha is None else float(alpha)
    lib.ot_ewald(float(L), a, int(nreal), int(nrecip), _p(p), int(p.shape[0]), _p(D), _p(g))
    return D, g


def ewald_hessian(points, L=1.0, alpha=None, nreal=4, nrecip=5):
    """O9 with second derivatives: (D[n], grad[n, 3], H[n, 6] in the order xx yy zz xy xz yz)."""
    lib = _load()
    p = np.ascontiguousarray(points, np.float64).reshape(-1, 3)
    D = np.empty(p.shape[0])
    g = np.empty((p.shape[0], 3))
    H = np.empty((p.shape[0], 6))
    a = 2.0 / L if alpha is None else float(alpha)
    lib.ot_ewald_hessian(float(L), a, int(nreal), int(nrecip), _p(p), int(p.shape[0]), _p(D), _p(g), _p(H))
    return D, g, H
