"""Handle bundle for one AMR grid: context, topology, moments and lists.

Pure marshalling over the C ABI (every step runs in libbh.so kernels).
"""
from __future__ import annotations

import torch

from . import binding as B


class BarnesHut:
    """Owns the library handles of one grid on one GPU.

    >>> bh = BarnesHut(grid)                      # topology, uploaded once
    >>> phi = bh.solve(rho, theta=0.5, precision=B.BH_FP32)
    """

    def __init__(self, grid, device: int = 0, group_cells: int = 64):
        self.device = device
        self.ctx = B.bh_ctx_create(device)
        self.grid = B.bh_grid_create_from(self.ctx, grid, group_cells)
        self.info = B.bh_grid_info(self.grid)
        self.m = None
        self.lists = None

    def close(self):
        if getattr(self, "lists", None) is not None:
            B.bh_lists_destroy(self.lists)
            self.lists = None
        if getattr(self, "m", None) is not None:
            B.bh_moments_destroy(self.m)
            self.m = None
        if getattr(self, "grid", None) is not None:
            B.bh_grid_destroy(self.grid)
            self.grid = None
        if getattr(self, "ctx", None) is not None:
            B.bh_ctx_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def sync_stream(self):
        B.bh_ctx_set_stream(self.ctx)

    def build_moments(self, rho: torch.Tensor):
        self.m = B.bh_build_moments(self.ctx, self.grid, rho, self.m)
        return self.m

    def walk(self, theta=0.5, theta_group=None, precision=B.BH_FP32):
        self.lists = B.bh_walk(self.ctx, self.grid, self.m, theta, theta_group, precision, self.lists)
        return self.lists

    def potential(self, phi: torch.Tensor, G=1.0, precision=B.BH_FP32):
        return B.bh_potential(self.ctx, self.grid, self.m, self.lists, G, precision, phi)

    def solve(self, rho: torch.Tensor, theta=0.5, theta_group=None, precision=B.BH_FP32, G=1.0, phi=None):
        """moments -> walk (lists) -> potential."""
        if phi is None:
            phi = torch.empty_like(rho)
        self.build_moments(rho)
        self.walk(theta, theta_group, precision)
        self.potential(phi, G, precision)
        return phi

    def solve_fused(self, rho: torch.Tensor, theta=0.5, theta_group=None, precision=B.BH_FP32, G=1.0, phi=None,
                    counts=None):
        """moments -> fused walk + potential (no lists, no host synchronisation)."""
        if phi is None:
            phi = torch.empty_like(rho)
        self.build_moments(rho)
        B.bh_walk_potential(self.ctx, self.grid, self.m, theta, theta_group, precision, G, phi, counts)
        return phi

    def solve_accel(self, rho: torch.Tensor, theta=0.5, theta_group=None, precision=B.BH_FP32, G=1.0, acc=None,
                    phi=None, counts=None):
        """moments -> fused walk + potential and acceleration sums; returns acc [n_leaf, 8, 8, 8, 3]
        (phi, if given, receives the potential of the same pass)."""
        if acc is None:
            acc = torch.empty(rho.shape + (3,), dtype=torch.float64, device=rho.device)
        self.build_moments(rho)
        B.bh_walk_accel(self.ctx, self.grid, self.m, theta, theta_group, precision, G, phi, acc, counts)
        return acc

    def solve_periodic(self, rho: torch.Tensor, table, theta=0.5, theta_group=None, precision=B.BH_FP32, G=1.0,
                       phi=None, counts=None):
        """moments -> periodic walk + potential (``table`` from bh_ewald_create for this grid's box)."""
        if phi is None:
            phi = torch.empty_like(rho)
        self.build_moments(rho)
        B.bh_walk_potential_periodic(self.ctx, self.grid, self.m, table, theta, theta_group, precision, G, phi,
                                     counts)
        return phi

    def direct_periodic(self, table, targets: torch.Tensor, G=1.0, out=None):
        if out is None:
            out = torch.empty(targets.numel(), dtype=torch.float64, device=targets.device)
        return B.bh_direct_periodic(self.ctx, self.grid, self.m, table, targets, G, out)

    def check(self):
        B.bh_moments_check(self.ctx, self.m)

    def direct(self, targets: torch.Tensor, G=1.0, out=None):
        if out is None:
            out = torch.empty(targets.numel(), dtype=torch.float64, device=targets.device)
        return B.bh_direct(self.ctx, self.grid, self.m, targets, G, out)

    def direct_accel(self, targets: torch.Tensor, G=1.0, out=None):
        if out is None:
            out = torch.empty((targets.numel(), 3), dtype=torch.float64, device=targets.device)
        return B.bh_direct_accel(self.ctx, self.grid, self.m, targets, G, out)

    # ---- host copies for tests and reports
    def node_keys(self):
        return B.bh_grid_node_keys(self.grid)

    def moments_host(self):
        return B.bh_moments_export(self.ctx, self.m, self.info["n_nodes"])

    def lists_host(self):
        return B.bh_lists_export(self.ctx, self.lists, self.info["n_groups"])
