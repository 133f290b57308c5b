"""Autotuner of the launch shape of one grid: group size and opening angle.

For each group size (32, 64, 128, 256, 512 cells) it finds the largest theta of
the grid {0.20, 0.25, ..., 1.00} whose RMS relative error against the exact
direct sum, on a seeded sample of cells, meets the target, times the whole
step (upward pass + fused walk and sums) at that theta, and keeps the
fastest.  The group size changes the result (the vote covers more or fewer
cells), which is why it is tuned under the error gate and not alone; the
traversal stack's depth limit and the tile of 64 nodes are fixed by the
wavefront width and need no tuning.  Everything numerical runs in libbh.so;
this module orders the calls and compares timings.
"""
from __future__ import annotations

import time

import numpy as np
import torch

from . import binding as B
from .solver import BarnesHut

GROUP_SIZES = (32, 64, 128, 256, 512)
THETA_GRID = np.round(np.arange(0.20, 1.0001, 0.05), 2)


def _timed(fn, reps):
    fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3 / reps


def tune_group_size(grid, rho: torch.Tensor, target: float, precision=B.BH_FP32, sample=None, direct=None,
                    sizes=GROUP_SIZES, reps=20, device=0, log=None):
    """Returns (best, table): best = dict(group_cells, theta, rms, ms) of the
    fastest group size meeting `target`; table = one such dict per size (theta
    None where no theta of the grid meets the target).  `sample`: canonical
    cell ids (int64 CUDA tensor; 1% seeded if None), `direct`: the exact
    potential there (computed if None)."""
    n = grid.ncells
    if sample is None:
        rng = np.random.default_rng(0)
        sample = torch.tensor(np.sort(rng.choice(n, max(1000, n // 100), replace=False)), dtype=torch.int64,
                              device=rho.device)
    table = []
    for G in sizes:
        bh = BarnesHut(grid, device=device, group_cells=G)
        if direct is None:
            bh.build_moments(rho)
            direct = bh.direct(sample)
        phi = torch.empty_like(rho)

        def step(theta, bh=bh, phi=phi):
            bh.build_moments(rho)
            B.bh_walk_potential(bh.ctx, bh.grid, bh.m, theta, None, precision, 1.0, phi, None)

        def rms(theta):
            step(theta)
            rel = (phi.reshape(-1).index_select(0, sample) - direct) / direct
            return float(torch.sqrt((rel * rel).mean()))

        found = None
        for th in THETA_GRID[::-1]:  # largest first: the first theta that meets the target is the one
            e = rms(float(th))
            if e <= target:
                found = (float(th), e)
                break
        row = dict(group_cells=G, theta=None, rms=None, ms=None)
        if found:
            row.update(theta=found[0], rms=found[1], ms=_timed(lambda: step(found[0]), reps))
        table.append(row)
        if log:
            log("group size %d: theta %s, sampled rms %s, %s ms" % (G, row["theta"], row["rms"], row["ms"]))
        bh.close()
    ok = [r for r in table if r["ms"] is not None]
    best = min(ok, key=lambda r: r["ms"]) if ok else None
    return best, table
