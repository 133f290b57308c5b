"""Batched solves: many grids in one persistent launch, queue orders, graph replay,
and the same for grids in one periodic box.

Each group is computed exactly as bh_walk_potential computes it, so every
grid's potential must equal its single-grid solve bit for bit, whatever the
queue order and however often a captured graph is replayed (with the
program's own eager work and synchronisations in between).
"""
import numpy as np
import pytest

from amr_inputs import maclaurin_spheroid, plummer_mix, random_amr, single_block, uniform_sphere

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1509_07370_amd import binding as B  # noqa: E402
from paper_1509_07370_amd.solver import BarnesHut  # noqa: E402


@pytest.fixture(scope="module")
def batch():
    grids = [single_block(seed=1), random_amr(5, nbase=2, max_level=2, zero_fraction=0.1), uniform_sphere(),
             maclaurin_spheroid(max_level=1), plummer_mix(7370, n_target_blocks=300), random_amr(6, nbase=1,
                                                                                                 max_level=3)]
    solvers = [BarnesHut(g) for g in grids]
    ctx = solvers[0].ctx
    # a batch needs all grids on one context
    handles = [B.bh_grid_create_from(ctx, g) for g in grids]
    b = B.bh_batch_create(ctx, handles)
    rho = [torch.tensor(g.rho, device="cuda") for g in grids]
    yield grids, solvers, ctx, handles, b, rho
    B.bh_batch_destroy(b)
    for h in handles:
        B.bh_grid_destroy(h)
    for s in solvers:
        s.close()


def _reference(solvers, rho, theta, precision):
    out = []
    for s, r in zip(solvers, rho):
        phi = torch.empty_like(r)
        s.solve_fused(r, theta, None, precision, 1.0, phi)
        out.append(phi)
    return out


@pytest.mark.parametrize("precision", [B.BH_FP32, B.BH_FP64])
def test_periodic_batch_equals_single_grid_solves(batch, precision):
    """bh_batch_solve_periodic: every grid of the batch in the same periodic box (side 1, one 33^3 table, its
    default budget for the group-centre cubics): potentials and counts equal bh_walk_potential_periodic's on each
    grid, bit for bit; a table of another box is refused."""
    grids, solvers, ctx, handles, b, rho = batch
    table = B.bh_ewald_create(ctx, 1.0, 33)
    ref, ref_counts = [], []
    for s_, r in zip(solvers, rho):
        t = B.bh_ewald_create(s_.ctx, 1.0, 33)
        phi = torch.empty_like(r)
        cn = torch.zeros((s_.info["n_groups"], 2), dtype=torch.int32, device="cuda")
        s_.solve_periodic(r, t, 0.6, None, precision, 1.0, phi, cn)
        torch.cuda.synchronize()
        B.bh_ewald_destroy(t)
        ref.append(phi)
        ref_counts.append(cn.cpu().numpy())
    phi = [torch.full_like(r, float("nan")) for r in rho]
    B.bh_batch_solve_periodic(ctx, b, table, rho, phi, 0.6, None, precision, 1.0)
    B.bh_batch_check(ctx, b)
    counts = B.bh_batch_counts(ctx, b)
    base = np.concatenate([[0], np.cumsum([c.shape[0] for c in ref_counts])])
    for k, (p, q) in enumerate(zip(phi, ref)):
        assert torch.equal(p, q), k
        assert np.array_equal(counts[base[k]:base[k + 1]], ref_counts[k]), k
    other = B.bh_ewald_create(ctx, 2.0, 9)
    with pytest.raises(B.BHError):
        B.bh_batch_solve_periodic(ctx, b, other, rho, phi, 0.6, None, precision, 1.0)
    B.bh_ewald_destroy(other)
    B.bh_ewald_destroy(table)


@pytest.mark.parametrize("precision", [B.BH_FP32, B.BH_FP64])
def test_batch_equals_single_grid_solves(batch, precision):
    grids, solvers, ctx, handles, b, rho = batch
    ref = _reference(solvers, rho, 0.6, precision)
    phi = [torch.full_like(r, float("nan")) for r in rho]
    B.bh_batch_solve(ctx, b, rho, phi, 0.6, None, precision, 1.0)
    B.bh_batch_check(ctx, b)
    for p, q in zip(phi, ref):
        assert torch.equal(p, q)


def test_cost_order_and_launch_width_do_not_change_results(batch):
    grids, solvers, ctx, handles, b, rho = batch
    ref = _reference(solvers, rho, 0.5, B.BH_FP32)
    phi = [torch.empty_like(r) for r in rho]
    B.bh_batch_solve(ctx, b, rho, phi, 0.5, None, B.BH_FP32, 1.0)
    counts = B.bh_batch_counts(ctx, b)
    assert counts.shape[0] == sum(s.info["n_groups"] for s in solvers) and counts[:, 0].sum() > 0
    B.bh_batch_schedule(ctx, b, B.BH_ORDER_COST)
    for per_cu in (1, 3, 0):
        B.bh_batch_set_launch(ctx, b, per_cu)
        for p in phi:
            p.fill_(float("nan"))
        B.bh_batch_solve(ctx, b, rho, phi, 0.5, None, B.BH_FP32, 1.0)
        for p, q in zip(phi, ref):
            assert torch.equal(p, q)
    B.bh_batch_schedule(ctx, b, B.BH_ORDER_NATURAL)


def test_graph_replays_match_eager(batch):
    grids, solvers, ctx, handles, b, rho = batch
    th = [None] * len(grids)
    th[2] = torch.full((solvers[2].info["n_groups"],), 0.8, dtype=torch.float32, device="cuda")
    phi = [torch.empty_like(r) for r in rho]
    B.bh_batch_solve(ctx, b, rho, phi, 0.7, th, B.BH_FP32, 1.0)
    eager = [p.clone() for p in phi]
    B.bh_batch_capture(ctx, b, rho, phi, 0.7, th, B.BH_FP32, 1.0)
    for rep in range(4):
        for p in phi:
            p.fill_(0.0)
        torch.cuda.synchronize()
        B.bh_batch_replay(ctx, b)
        torch.cuda.synchronize()
        for p, q in zip(phi, eager):
            assert torch.equal(p, q), rep
        _ = (rho[0] * 2).sum().item()  # eager work between replays
    B.bh_batch_check(ctx, b)


def test_invalid_density_is_reported_per_replay(batch):
    grids, solvers, ctx, handles, b, rho = batch
    bad = [r.clone() for r in rho]
    bad[3][0, 0, 0, 0] = -1.0
    phi = [torch.empty_like(r) for r in rho]
    B.bh_batch_solve(ctx, b, bad, phi, 0.5, None, B.BH_FP32, 1.0)
    with pytest.raises(B.BHError) as ei:
        B.bh_batch_check(ctx, b)
    assert ei.value.code == B.BH_EINVAL and "grid 3" in str(ei.value)
    B.bh_batch_solve(ctx, b, rho, phi, 0.5, None, B.BH_FP32, 1.0)
    B.bh_batch_check(ctx, b)


def test_launch_configurations_and_autotuner(batch):
    """Order, width and kernel variant keep the bits; a lower stack limit keeps
    the far/near sets (counts) and changes only the summation order."""
    grids, solvers, ctx, handles, b, rho = batch
    ref = _reference(solvers, rho, 0.7, B.BH_FP32)
    phi = [torch.empty_like(r) for r in rho]
    B.bh_batch_solve(ctx, b, rho, phi, 0.7, None, B.BH_FP32, 1.0)
    ref_counts = B.bh_batch_counts(ctx, b)
    for cfg in (dict(order=B.BH_ORDER_COST, workgroups_per_cu=2, waves_per_simd=4, stack_limit=0),
                dict(order=B.BH_ORDER_NATURAL, workgroups_per_cu=0, waves_per_simd=6, stack_limit=0),
                dict(order=B.BH_ORDER_COST, workgroups_per_cu=1, waves_per_simd=8, stack_limit=0),
                dict(order=B.BH_ORDER_NATURAL, workgroups_per_cu=3, waves_per_simd=8, stack_limit=8),
                dict(order=B.BH_ORDER_COST, workgroups_per_cu=0, waves_per_simd=6, stack_limit=64)):
        B.bh_batch_configure(ctx, b, **cfg)
        assert B.bh_batch_get_config(b) == cfg
        for p in phi:
            p.fill_(float("nan"))
        B.bh_batch_solve(ctx, b, rho, phi, 0.7, None, B.BH_FP32, 1.0)
        B.bh_batch_check(ctx, b)
        assert np.array_equal(B.bh_batch_counts(ctx, b), ref_counts)
        for p, q in zip(phi, ref):
            if cfg["stack_limit"] == 0:
                assert torch.equal(p, q)
            else:
                assert float(((p - q) / q).abs().max()) <= 1e-5
    # fp64 variants; an fp32-only variant is refused for an fp64 solve
    ref64 = _reference(solvers, rho, 0.7, B.BH_FP64)
    for waves in (2, 4):
        B.bh_batch_configure(ctx, b, waves_per_simd=waves)
        B.bh_batch_solve(ctx, b, rho, phi, 0.7, None, B.BH_FP64, 1.0)
        for p, q in zip(phi, ref64):
            assert torch.equal(p, q)
    B.bh_batch_configure(ctx, b, waves_per_simd=6)
    with pytest.raises(B.BHError):
        B.bh_batch_solve(ctx, b, rho, phi, 0.7, None, B.BH_FP64, 1.0)
    for bad in (dict(waves_per_simd=5), dict(stack_limit=4), dict(order=7), dict(workgroups_per_cu=65)):
        with pytest.raises(B.BHError):
            B.bh_batch_configure(ctx, b, **bad)
    # the autotuner tries every candidate and leaves the best one applied
    best, best_ms, table = B.bh_batch_autotune(ctx, b, rho, phi, 0.7, None, B.BH_FP32, 1.0, reps=1)
    assert len(table) == 36 and best_ms > 0
    assert best_ms == min(t for _, t in table)
    assert B.bh_batch_get_config(b) == best
    B.bh_batch_solve(ctx, b, rho, phi, 0.7, None, B.BH_FP32, 1.0)
    B.bh_batch_check(ctx, b)
    for p, q in zip(phi, ref):
        assert float(((p - q) / q).abs().max()) <= 1e-5
    B.bh_batch_configure(ctx, b)
