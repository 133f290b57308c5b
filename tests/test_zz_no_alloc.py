"""bh_potential_static (no device allocation, static scratch) against
bh_build_moments + bh_walk_potential, through the C ABI.

* two calls in a row on one GPU, the second on a smaller grid: every
  potential and every group's counts equal the two-call path's, bit for bit,
  in fp64 and fp32, with one theta and with a per-group theta array;
* the status words report an invalid density and are cleared by the next call;
* a grid whose workspace exceeds the static scratch is refused before any work.
"""
import numpy as np
import pytest

from amr_inputs import maclaurin_spheroid, random_amr, uniform_sphere

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1509_07370_amd import binding as B  # noqa: E402
from paper_1509_07370_amd.solver import BarnesHut  # noqa: E402


def _reference(bh, rho, theta, theta_group, precision):
    phi = torch.empty_like(rho)
    counts = torch.zeros((bh.info["n_groups"], 2), dtype=torch.int32, device="cuda")
    bh.build_moments(rho)
    B.bh_walk_potential(bh.ctx, bh.grid, bh.m, theta, theta_group, precision, 1.5, phi, counts)
    bh.check()
    return phi, counts


def _static(bh, rho, theta, theta_group, precision):
    phi = torch.full_like(rho, float("nan"))
    counts = torch.full((bh.info["n_groups"], 2), -1, dtype=torch.int32, device="cuda")
    status = torch.full((2,), 7, dtype=torch.int32, device="cuda")
    B.bh_potential_static(bh.ctx, bh.grid, rho, theta, theta_group, precision, 1.5, phi, counts, status)
    torch.cuda.synchronize()
    return phi, counts, status


@pytest.mark.parametrize("precision", [B.BH_FP32, B.BH_FP64])
def test_two_calls_match_the_two_call_path(precision):
    big = maclaurin_spheroid(max_level=2)       # 4.5e5 cells
    small = random_amr(21, nbase=2, max_level=2, p_refine=0.3, zero_fraction=0.1)
    cases = []
    for g in (big, small):
        bh = BarnesHut(g)
        rho = torch.tensor(g.rho, device="cuda")
        cases.append((g, bh, rho))
    # both grids run through the scratch before the comparisons, so the second
    # (smaller) call starts from what the first left behind
    results = []
    for k, (g, bh, rho) in enumerate(cases):
        ng = bh.info["n_groups"]
        th = torch.tensor(np.random.default_rng(k).uniform(0.3, 1.0, ng).astype(np.float32), device="cuda")
        for theta, tg in ((0.7, None), (0.5, th)):
            results.append((bh, rho, theta, tg) + _static(bh, rho, theta, tg, precision))
    for bh, rho, theta, tg, phi, counts, status in results:
        ref, ref_counts = _reference(bh, rho, theta, tg, precision)
        assert torch.equal(phi, ref)
        assert torch.equal(counts, ref_counts)
        assert status.cpu().tolist() == [0, 0]
    for _, bh, _ in cases:
        bh.close()


def test_status_reports_invalid_density_and_is_cleared():
    g = random_amr(5, nbase=2, max_level=1, p_refine=0.3)
    bh = BarnesHut(g)
    rho = torch.tensor(g.rho, device="cuda")
    bad = rho.clone()
    bad[2, 1, 3, 4] = -1.0
    _, _, status = _static(bh, bad, 0.6, None, B.BH_FP32)
    assert status.cpu().tolist()[0] != 0
    phi, counts, status = _static(bh, rho, 0.6, None, B.BH_FP32)
    assert status.cpu().tolist() == [0, 0]
    ref, ref_counts = _reference(bh, rho, 0.6, None, B.BH_FP32)
    assert torch.equal(phi, ref) and torch.equal(counts, ref_counts)
    # without a status array the call still runs
    phi2 = torch.empty_like(rho)
    B.bh_potential_static(bh.ctx, bh.grid, rho, 0.6, None, B.BH_FP32, 1.5, phi2, None, None)
    assert torch.equal(phi2, ref)
    bh.close()


def test_grid_beyond_the_scratch_is_refused():
    g = uniform_sphere(nbase=16)  # 4096 blocks, 2.1M cells: about 170 MB of workspace
    bh = BarnesHut(g)
    rho = torch.ones(g.rho.shape, dtype=torch.float64, device="cuda")
    phi = torch.zeros_like(rho)
    with pytest.raises(B.BHError) as ei:
        B.bh_potential_static(bh.ctx, bh.grid, rho, 0.5, None, B.BH_FP32, 1.0, phi, None, None)
    assert ei.value.code == B.BH_ECAPACITY and "static scratch" in str(ei.value)
    torch.cuda.synchronize()
    assert bool((phi == 0).all())
    with pytest.raises(B.BHError) as ei:
        B.bh_potential_static(bh.ctx, bh.grid, rho, 1.5, None, B.BH_FP32, 1.0, phi, None, None)
    assert ei.value.code == B.BH_EINVAL
    bh.close()
