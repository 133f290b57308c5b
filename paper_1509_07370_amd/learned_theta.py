"""Learned per-group opening angle: labels, training and inference.

Everything numerical runs in libbh.so kernels (walk + sums, direct sum,
per-group error, features, network forward / gradient / Adam); this module
only orders the calls and keeps small host-side bookkeeping (label envelope,
mini-batch order, files).

Labels come from the method itself, from tables of every group's RMS relative
error against the exact direct sum and of its far/near counts at each theta of
the grid {0.20, 0.25, ..., 1.00}:
  * "target": the largest theta whose error, and the error of every smaller
    theta, meets the target (each group on its own);
  * "lagrange": the cost-aware split of one error budget over the groups,
    theta_g = argmin_theta cost_g(theta) + lambda err_g(theta)^2, with cost_g the
    group's walk time from a linear model of the counts (fitted to timed
    sweeps) and lambda, per training grid, the smallest multiplier that makes
    that grid's global RMS meet the target: each label is the group's theta in
    the cheapest allocation that brings its own grid to the target.
A network keeps the smallest label it was trained on as its theta floor
(bh_mlp_set_theta_floor): under it the network extrapolates, and a group pushed
there by the output shift walks far longer than the rest.  A network may be
trained for another opening test or far-field order of bh_walk_potential_ex
(the walk options, kept in its metadata with the floor).
At run time the network's bf16 output drives bh_walk_potential; a 1% sample of
cells is checked against the direct sum and a fixed conservative theta (0.4)
is used instead if the sample misses the target.  calibrate_on_sample picks
the network's output shift for one grid from the same sample (the analogue of
choosing a fixed theta by a sweep).

Usage on a GPU:
  python -m paper_1509_07370_amd.learned_theta train --target 1e-3 --out paper_1509_07370_amd/data/theta_mlp_1e-3.npz
  python -m paper_1509_07370_amd.learned_theta train --target 1e-4 --labels lagrange \
      --out paper_1509_07370_amd/data/theta_mlp_lagrange_1e-4.npz
  python -m paper_1509_07370_amd.learned_theta train --target 1e-3 --labels lagrange --opening group_box --order 0 \
      --out paper_1509_07370_amd/data/theta_mlp_paper_lagrange_1e-3.npz
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np
import torch

from . import binding as B
from .solver import BarnesHut

THETA_GRID = np.round(np.arange(0.20, 1.0001, 0.05), 2)
DEFAULT_WALK = (B.BH_MAC_CELLS, 2)  # (opening test, far-field order) of bh_walk_potential
OPENING = {"cells": B.BH_MAC_CELLS, "group_box": B.BH_MAC_GROUP_BOX}


def walk(bh, theta, theta_group, precision, G, phi, counts=None, options=DEFAULT_WALK):
    """bh_walk_potential, or bh_walk_potential_ex for another opening test / far-field order."""
    if tuple(options) == DEFAULT_WALK:
        B.bh_walk_potential(bh.ctx, bh.grid, bh.m, theta, theta_group, precision, G, phi, counts)
    else:
        B.bh_walk_potential_ex(bh.ctx, bh.grid, bh.m, theta, theta_group, precision, G, phi, counts,
                               mac=options[0], order=options[1])


def learned_walk(bh, net, shift, precision, G, phi, theta, counts=None):
    """The network's per-group thetas (into ``theta``), then the walk with them: the one fused call for the
    default walk, bh_theta_infer then bh_walk_potential_ex for other walk options."""
    if net.walk_options == DEFAULT_WALK:
        B.bh_learned_walk_potential(bh.ctx, bh.grid, bh.m, net.h, float(shift), precision, G, phi, theta, counts)
    else:
        B.bh_theta_infer(bh.ctx, bh.grid, bh.m, net.h, theta, float(shift))
        walk(bh, 0.5, theta, precision, G, phi, counts, net.walk_options)
FALLBACK_THETA = 0.4
DATA_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "data")


def direct_potential(bh: BarnesHut, rho: torch.Tensor) -> torch.Tensor:
    """Exact fp64 direct sum at every cell (GPU), caller layout."""
    bh.build_moments(rho)
    n = bh.info["n_cells"]
    return bh.direct(torch.arange(n, device=rho.device, dtype=torch.int64)).reshape(rho.shape)


def error_table(bh: BarnesHut, rho: torch.Tensor, direct: torch.Tensor, thetas=THETA_GRID,
                precision=B.BH_FP32, options=DEFAULT_WALK) -> np.ndarray:
    """[len(thetas), n_groups] per-group RMS relative error of the walk at each theta."""
    ng = bh.info["n_groups"]
    bh.build_moments(rho)
    phi = torch.empty_like(rho)
    rms = torch.empty((len(thetas), ng), dtype=torch.float32, device=rho.device)
    for k, th in enumerate(thetas):
        walk(bh, float(th), None, precision, 1.0, phi, None, options)
        B.bh_group_rms_error(bh.ctx, bh.grid, phi, direct, rms[k])
    bh.check()
    return rms.cpu().numpy()


def count_table(bh: BarnesHut, rho: torch.Tensor, thetas=THETA_GRID, precision=B.BH_FP32, reps=5,
                options=DEFAULT_WALK):
    """[len(thetas), n_groups, 2] far / near counts of every group at each theta, and the timed step (moments +
    fused walk and sums) in ms at each theta."""
    ng = bh.info["n_groups"]
    phi = torch.empty_like(rho)
    cn = torch.zeros((ng, 2), dtype=torch.int32, device=rho.device)
    counts = np.empty((len(thetas), ng, 2), np.int32)
    ms = np.empty(len(thetas))
    for k, th in enumerate(thetas):
        def step(th=float(th)):
            bh.build_moments(rho)
            walk(bh, th, None, precision, 1.0, phi, None, options)
        step()
        walk(bh, float(th), None, precision, 1.0, phi, cn, options)
        counts[k] = cn.cpu().numpy()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            step()
        torch.cuda.synchronize()
        ms[k] = (time.perf_counter() - t0) * 1e3 / reps
    return counts, ms


def fit_time_model(counts_per_grid, ms_per_grid):
    """Least-squares ms = a * sum(far) + b * sum(near) + c over every (grid, theta): per-entry walk times."""
    rows, y = [], []
    for c, ms in zip(counts_per_grid, ms_per_grid):
        for k in range(c.shape[0]):
            rows.append([c[k, :, 0].sum(), c[k, :, 1].sum(), 1.0])
            y.append(ms[k])
    coef, *_ = np.linalg.lstsq(np.array(rows, np.float64), np.array(y), rcond=None)
    return float(coef[0]), float(coef[1]), float(coef[2])


def lagrangian_labels(errs: np.ndarray, counts: np.ndarray, model, lam: float, thetas=THETA_GRID) -> np.ndarray:
    """theta_g = argmin over the grid of cost_g(theta) + lam * err_g(theta)^2 (cost in ms from the time model)."""
    a, b, _ = model
    J = a * counts[:, :, 0] + b * counts[:, :, 1] + lam * errs.astype(np.float64) ** 2
    return np.asarray(thetas)[np.argmin(J, axis=0)].astype(np.float32)


def lambda_for_target(errs: np.ndarray, counts: np.ndarray, model, target: float, thetas=THETA_GRID) -> float:
    """Smallest multiplier whose labels give the grid a global RMS within the target (bisection in log lambda)."""
    lo, hi = 1e-12, 1e12
    for _ in range(120):
        mid = float(np.sqrt(lo * hi))
        if estimated_rms(errs, lagrangian_labels(errs, counts, model, mid, thetas), thetas) <= target:
            hi = mid
        else:
            lo = mid
    return hi


def labels_from_errors(errs: np.ndarray, target: float, thetas=THETA_GRID) -> np.ndarray:
    """Largest theta whose error, and the error of every smaller theta, meets the target."""
    ok = np.logical_and.accumulate(errs <= target, axis=0)
    k = ok.sum(axis=0) - 1
    return np.asarray(thetas)[np.maximum(k, 0)].astype(np.float32)


def group_features(bh: BarnesHut, rho: torch.Tensor, out=None) -> torch.Tensor:
    bh.build_moments(rho)
    if out is None:
        out = torch.empty((bh.info["n_groups"], B.MLP_INPUTS), dtype=torch.float32, device=rho.device)
    return B.bh_group_features(bh.ctx, bh.grid, bh.m, out)


class ThetaNet:
    """Handle of one bh_mlp network plus its input normalisation."""

    def __init__(self, ctx, params, mean, scale, meta=None):
        self.ctx = ctx
        self.mean = np.asarray(mean, np.float32)
        self.scale = np.asarray(scale, np.float32)
        self.h = B.bh_mlp_create(ctx, params, self.mean, self.scale)
        self.meta = dict(meta or {})
        if "theta_floor" in self.meta:
            B.bh_mlp_set_theta_floor(ctx, self.h, self.meta["theta_floor"])

    @classmethod
    def fresh(cls, ctx, feat_host: np.ndarray, params, meta=None):
        mean = feat_host.mean(0)
        std = feat_host.std(0)
        scale = 1.0 / np.maximum(std, 1e-3)
        return cls(ctx, params, mean, scale, meta)

    def close(self):
        if getattr(self, "h", None) is not None:
            B.bh_mlp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def params(self) -> np.ndarray:
        return B.bh_mlp_get_params(self.ctx, self.h)

    @property
    def shift(self) -> float:
        return float(self.meta.get("theta_shift", 0.0))

    @property
    def floor(self) -> float:
        """Smallest theta the inference returns (the smallest training label; 0.2 for older networks)."""
        return float(self.meta.get("theta_floor", 0.2))

    @property
    def walk_options(self):
        """(opening test, far-field order) of the walk the network was trained for."""
        return (int(self.meta.get("mac", DEFAULT_WALK[0])), int(self.meta.get("order", DEFAULT_WALK[1])))

    def predict(self, feat: torch.Tensor, bf16=True, out=None, shift=None) -> torch.Tensor:
        if out is None:
            out = torch.empty(feat.shape[0], dtype=torch.float32, device=feat.device)
        return B.bh_mlp_forward(self.ctx, self.h, feat, out, bf16, self.shift if shift is None else shift)

    def train(self, feat: torch.Tensor, label: torch.Tensor, epochs=200, batch=4096, lr=3e-3, seed=42, log=None):
        """Adam on mini-batches of the mean squared error; returns per-epoch mean loss."""
        n = feat.shape[0]
        gen = torch.Generator(device="cpu").manual_seed(seed)
        grad = torch.empty(B.MLP_PARAMS, dtype=torch.float32, device=feat.device)
        loss = torch.zeros(1, dtype=torch.float32, device=feat.device)
        hist = []
        for ep in range(epochs):
            perm = torch.randperm(n, generator=gen).to(feat.device)
            tot = torch.zeros((), dtype=torch.float32, device=feat.device)
            nb = 0
            for b0 in range(0, n, batch):
                idx = perm[b0:b0 + batch]
                xb = feat.index_select(0, idx).contiguous()
                yb = label.index_select(0, idx).contiguous()
                B.bh_mlp_grad(self.ctx, self.h, xb, yb, grad, loss)
                B.bh_mlp_adam_step(self.ctx, self.h, grad, lr)
                tot += loss[0]
                nb += 1
            hist.append(float(tot) / nb)
            if log and (ep % max(1, epochs // 10) == 0 or ep == epochs - 1):
                log("epoch %d loss %.3e" % (ep, hist[-1]))
        return hist

    def save(self, path):
        os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
        np.savez(path, params=self.params(), mean=self.mean, scale=self.scale,
                 meta=np.array(json.dumps(self.meta)))

    @classmethod
    def load(cls, ctx, path):
        z = np.load(path, allow_pickle=False)
        return cls(ctx, z["params"], z["mean"], z["scale"], json.loads(str(z["meta"])))


def solve_learned(bh: BarnesHut, rho: torch.Tensor, net: ThetaNet, phi: torch.Tensor, feat: torch.Tensor,
                  theta: torch.Tensor, precision=B.BH_FP32, G=1.0):
    """moments, then bh_learned_walk_potential: per group features + bf16 network (one kernel), then the walk +
    sums with those thetas (the thetas used land in ``theta``).  ``feat`` is unused (kept for callers that
    stage features)."""
    bh.build_moments(rho)
    learned_walk(bh, net, net.shift, precision, G, phi, theta)
    return phi


def solve_learned_two_step(bh: BarnesHut, rho: torch.Tensor, net: ThetaNet, phi: torch.Tensor, theta: torch.Tensor,
                           precision=B.BH_FP32, G=1.0):
    """The same step in two launches: bh_theta_infer, then bh_walk_potential with the theta array."""
    bh.build_moments(rho)
    B.bh_theta_infer(bh.ctx, bh.grid, bh.m, net.h, theta, net.shift)
    walk(bh, 0.5, theta, precision, G, phi, None, net.walk_options)
    return phi


def sampled_rms(bh: BarnesHut, phi: torch.Tensor, frac=0.01, seed=0, minimum=1000) -> float:
    """RMS relative error of phi against the exact direct sum on a seeded sample of cells."""
    n = bh.info["n_cells"]
    k = min(n, max(minimum, int(frac * n)))
    rng = np.random.default_rng(seed)
    tg = torch.tensor(np.sort(rng.choice(n, k, replace=False)), dtype=torch.int64, device=phi.device)
    d = bh.direct(tg)
    rel = (phi.reshape(-1).index_select(0, tg) - d) / d
    return float(torch.sqrt((rel * rel).mean()))


def calibrate_on_sample(bh, rho, net, phi, theta, target, precision=B.BH_FP32, margin=0.95,
                        shifts=np.round(np.arange(-0.3, 0.6001, 0.025), 3), frac=0.01, seed=0):
    """The smallest output shift whose learned step meets margin * target on a seeded 1% sample of cells against
    the exact direct sum (None if none does).  Sets net.meta['theta_shift'] to it and returns it."""
    n = bh.info["n_cells"]
    k = min(n, max(1000, int(frac * n)))
    rng = np.random.default_rng(seed)
    tg = torch.tensor(np.sort(rng.choice(n, k, replace=False)), dtype=torch.int64, device=phi.device)
    bh.build_moments(rho)
    d = bh.direct(tg)
    for s_ in shifts:
        bh.build_moments(rho)
        learned_walk(bh, net, s_, precision, 1.0, phi, theta)
        rel = (phi.reshape(-1).index_select(0, tg) - d) / d
        if float(torch.sqrt((rel * rel).mean())) <= margin * target:
            net.meta["theta_shift"] = float(s_)
            return float(s_)
    return None


def solve_with_fallback(bh, rho, net, phi, feat, theta, target, precision=B.BH_FP32, G=1.0):
    """Learned theta, judged by a 1% sampled direct sum; fixed theta 0.4 if it misses the target."""
    solve_learned(bh, rho, net, phi, feat, theta, precision, G)
    err = sampled_rms(bh, phi)
    if err <= target:
        return phi, dict(mode="learned", sampled_rms=err)
    walk(bh, FALLBACK_THETA, None, precision, G, phi, None, net.walk_options)
    return phi, dict(mode="fallback", sampled_rms_learned=err, sampled_rms=sampled_rms(bh, phi))


# ------------------------------------------------------------------ training workloads

def training_grids(extended=False):
    """Seeded perturbations of the uniform-sphere and MacLaurin workloads; `extended` adds
    3-level meshes shaped like the held-out cores (e in {0.7, 0.8, 0.9, 0.95}, a1 in {0.2, 0.3})
    and two 3-level spheres."""
    from amr_inputs import maclaurin_spheroid, uniform_sphere
    out = []
    for e in (0.75, 0.85, 0.9, 0.95):
        for a1 in (0.2, 0.3):
            out.append(maclaurin_spheroid(e=e, a1=a1, max_level=2))
    out.append(maclaurin_spheroid(e=0.8, a1=0.25, max_level=3))
    for R in (0.25, 0.4):
        for ro in (1e-3, 1e-5):
            out.append(uniform_sphere(radius=R, rho_out=ro, max_level=2))
    if extended:
        out += [maclaurin_spheroid(e=e, a1=a1, max_level=3) for e in (0.7, 0.8, 0.9, 0.95) for a1 in (0.2, 0.3)]
        out += [uniform_sphere(radius=R, rho_out=1e-4, max_level=3) for R in (0.2, 0.3)]
    return out


def evaluation_grids(seed=2024, count=3):
    """Held-out MacLaurin cores shaped like the benchmark workload (e in [0.7, 0.95])."""
    from amr_inputs import maclaurin_spheroid
    rng = np.random.default_rng(seed)
    return [maclaurin_spheroid(e=float(e), a1=0.25, max_level=3) for e in rng.uniform(0.7, 0.95, count)]


def estimated_rms(errs: np.ndarray, theta: np.ndarray, thetas=THETA_GRID) -> float:
    """Global RMS error of one grid if group g walks with theta[g], estimated
    from its error table at the smallest tabulated theta >= theta[g]."""
    k = np.clip(np.searchsorted(np.asarray(thetas), np.asarray(theta) - 1e-6), 0, len(thetas) - 1)
    e = errs[k, np.arange(errs.shape[1])]
    return float(np.sqrt(np.mean(e.astype(np.float64) ** 2)))


def calibrate_shift(net, feats_per_grid, errs_per_grid, target, shifts=np.arange(0.0, 0.5001, 0.025)):
    """Smallest output shift for which every training grid meets the target."""
    for s in shifts:
        ok = True
        for f, e in zip(feats_per_grid, errs_per_grid):
            th = net.predict(torch.tensor(f, device="cuda"), bf16=True, shift=float(s)).cpu().numpy()
            th = np.maximum(th, net.floor)
            if estimated_rms(e, th) > target:
                ok = False
                break
        if ok:
            return float(s)
    return float(shifts[-1])


def build_dataset(grids, target, log=print, labels="target", options=DEFAULT_WALK):
    feats, labs, errs, counts, times = [], [], [], [], []
    for g in grids:
        t0 = time.time()
        bh = BarnesHut(g)
        rho = torch.tensor(g.rho, device="cuda")
        direct = direct_potential(bh, rho)
        table = error_table(bh, rho, direct, options=options)
        f = group_features(bh, rho).cpu().numpy()
        feats.append(f)
        errs.append(table)
        if labels == "lagrange":
            c, ms = count_table(bh, rho, options=options)
            counts.append(c)
            times.append(ms)
        else:
            labs.append(labels_from_errors(table, target))
        log("data %s: %d groups, %.1f s" % (g.name, f.shape[0], time.time() - t0))
        bh.close()
    info = {}
    if labels == "lagrange":
        model = fit_time_model(counts, times)
        lams = [lambda_for_target(e, c, model, target) for e, c in zip(errs, counts)]
        labs = [lagrangian_labels(e, c, model, lam) for e, c, lam in zip(errs, counts, lams)]
        info = dict(time_model=model, grid_lams=lams)
        log("time model: %.3e ms per far entry, %.3e per near entry, %.3f ms fixed; lambda per grid %s" % (
            model[0], model[1], model[2], np.round(lams, 1).tolist()))
    for y in labs:
        log("mean label %.3f" % y.mean())
    return feats, labs, errs, info


def evaluate(net: ThetaNet, grids, target, precision=B.BH_FP32, reps=10, log=print):
    """Learned theta vs every fixed theta of the grid on held-out workloads."""
    out = []
    for g in grids:
        bh = BarnesHut(g)
        rho = torch.tensor(g.rho, device="cuda")
        direct = direct_potential(bh, rho)
        ng = bh.info["n_groups"]
        n = bh.info["n_cells"]
        phi = torch.empty_like(rho)
        feat = torch.empty((ng, B.MLP_INPUTS), dtype=torch.float32, device="cuda")
        theta = torch.empty(ng, dtype=torch.float32, device="cuda")

        def rms_of(p):
            rel = ((p - direct) / direct).reshape(-1)
            return float(torch.sqrt((rel * rel).mean()))

        def timed(fn):
            fn()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                fn()
            torch.cuda.synchronize()
            return (time.perf_counter() - t0) * 1e3 / reps

        fixed = []
        for th in THETA_GRID:
            def run(th=float(th)):
                bh.build_moments(rho)
                walk(bh, th, None, precision, 1.0, phi, None, net.walk_options)
            ms = timed(run)
            fixed.append(dict(theta=float(th), rms=rms_of(phi), ms=ms))
        ms_l = timed(lambda: solve_learned(bh, rho, net, phi, feat, theta, precision))
        th = theta.cpu().numpy()
        rec = dict(grid=g.name, meta={k: v for k, v in g.meta.items() if k in ("e", "a1")}, cells=n,
                   learned=dict(rms=rms_of(phi), ms=ms_l, mcells=n / ms_l / 1e3, theta_mean=float(th.mean()),
                                theta_p10=float(np.percentile(th, 10)), theta_p90=float(np.percentile(th, 90)),
                                sampled_rms=sampled_rms(bh, phi), shift=net.shift),
                   fixed=fixed)
        # the shift chosen for this grid on its own 1% sample
        stored = net.shift
        s_ = calibrate_on_sample(bh, rho, net, phi, theta, target, precision)
        if s_ is not None:
            ms_c = timed(lambda: solve_learned(bh, rho, net, phi, feat, theta, precision))
            rec["learned_calibrated"] = dict(shift=s_, rms=rms_of(phi), ms=ms_c, mcells=n / ms_c / 1e3)
        net.meta["theta_shift"] = stored
        ok = [f for f in fixed if f["rms"] <= target]
        best = max(ok, key=lambda f: f["theta"]) if ok else None
        rec["best_fixed"] = best
        if best:
            rec["learned_speedup_vs_best_fixed"] = best["ms"] / ms_l
            if "learned_calibrated" in rec:
                rec["calibrated_speedup_vs_best_fixed"] = best["ms"] / rec["learned_calibrated"]["ms"]
        log("eval e=%.3f: learned rms %.2e %.3f ms (theta mean %.3f) | best fixed theta %s rms %s %s ms" % (
            g.meta.get("e", 0), rec["learned"]["rms"], ms_l, th.mean(), best and best["theta"],
            best and "%.2e" % best["rms"], best and "%.3f" % best["ms"]))
        if "learned_calibrated" in rec:
            c = rec["learned_calibrated"]
            log("    calibrated on the 1%% sample: shift %.3f, rms %.2e, %.3f ms (x%.3f vs best fixed)" % (
                c["shift"], c["rms"], c["ms"], rec.get("calibrated_speedup_vs_best_fixed", float("nan"))))
        out.append(rec)
        bh.close()
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("cmd", choices=["train", "evaluate"])
    ap.add_argument("--weights", default=None)
    ap.add_argument("--target", default="1e-3", help="RMS target, as it appears in the weights file name")
    ap.add_argument("--epochs", type=int, default=300)
    ap.add_argument("--lr", type=float, default=3e-3)
    ap.add_argument("--out", default=None)
    ap.add_argument("--labels", choices=["target", "lagrange"], default="target")
    ap.add_argument("--extended", action="store_true", help="add the 3-level training meshes")
    ap.add_argument("--opening", choices=sorted(OPENING), default="cells",
                    help="opening test of the walk the labels come from (bh_walk_potential_ex)")
    ap.add_argument("--order", type=int, choices=[0, 2], default=2, help="far-field order of that walk")
    args = ap.parse_args(argv)
    from amr_inputs.mlp_init import glorot_init

    def log(msg):
        print("[learned-theta] " + msg, flush=True)

    ctx = B.bh_ctx_create(0)
    if args.cmd == "evaluate":
        net = ThetaNet.load(ctx, args.weights or os.path.join(DATA_DIR, "theta_mlp_%s.npz" % args.target))
        res = evaluate(net, evaluation_grids(), float(net.meta.get("target", float(args.target))), log=log)
        print(json.dumps(dict(target=net.meta.get("target"), shift=net.shift, results=res)))
        return 0
    target = float(args.target)
    options = (OPENING[args.opening], args.order)
    F, Y, E, info = build_dataset(training_grids(args.extended), target, log, labels=args.labels, options=options)
    X, y = np.concatenate(F), np.concatenate(Y)
    net = ThetaNet.fresh(ctx, X, glorot_init(42).astype(np.float32),
                         meta=dict(target=target, epochs=args.epochs, lr=args.lr, n_train=int(len(y)), seed=42,
                                   labels=args.labels, extended=bool(args.extended),
                                   theta_floor=float(y.min()), mac=int(options[0]), order=int(options[1]),
                                   **{k: v for k, v in info.items() if k in ("time_model", "grid_lams")}))
    fx = torch.tensor(X, device="cuda")
    fy = torch.tensor(y, device="cuda")
    t0 = time.time()
    hist = net.train(fx, fy, epochs=args.epochs, lr=args.lr, log=log)
    net.meta.update(final_loss=hist[-1], train_seconds=time.time() - t0)
    pred = net.predict(fx, bf16=True).cpu().numpy()
    log("train mse %.3e, mean |pred - label| %.3f, label mean %.3f" % (
        float(np.mean((pred - y) ** 2)), float(np.mean(np.abs(pred - y))), float(y.mean())))
    net.meta["theta_shift"] = calibrate_shift(net, F, E, target)
    log("calibrated output shift %.3f" % net.meta["theta_shift"])
    out = args.out or os.path.join(DATA_DIR, "theta_mlp_%s.npz" % args.target)
    net.save(out)
    log("saved " + out)
    return 0


if __name__ == "__main__":
    sys.exit(main())
