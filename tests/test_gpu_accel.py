"""Accelerations g = -grad phi on the GPU vs the CPU oracle, through the C ABI.

* bh_walk_accel against the oracle's walk + O8 sums, cell by cell, on every
  group without a marginal decision (fp64 within 1e-12, fp32 within 1e-5 of
  the cell's scale), with identical far/near counts there; its potential
  output within the potential path's tolerances;
* bh_direct_accel within 1e-12 of the oracle's direct acceleration;
* a theta small enough to open every node reproduces the direct acceleration;
* invalid arguments are refused.

Scale of a cell: max(|g_ref|, 0.1 RMS |g_ref| over the grid), so that cells
where the field nearly cancels are judged against the field's size.
"""
import numpy as np
import pytest

from amr_inputs import maclaurin_spheroid, random_amr, single_block, uniform_sphere
from oracle import OracleTree
from oracle.oracle import fp32_band_for

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1509_07370_amd import binding as B  # noqa: E402
from paper_1509_07370_amd.solver import BarnesHut  # noqa: E402

# fp32: the band derived from fp32 rounding (every test grid lies in the unit box)
TAU = {B.BH_FP64: 1e-12, B.BH_FP32: fp32_band_for(1.0)}
TOL = {B.BH_FP64: 1e-12, B.BH_FP32: 1e-5}

GRIDS = {
    "single_block": lambda: single_block(seed=3, sigma=1.0),
    "random_amr": lambda: random_amr(21, nbase=2, max_level=3, p_refine=0.3, zero_fraction=0.1),
    "sphere": lambda: uniform_sphere(),
    "maclaurin_l1": lambda: maclaurin_spheroid(max_level=1),
}
_cache = {}


def setup(name):
    if name not in _cache:
        g = GRIDS[name]()
        bh = BarnesHut(g)
        rho = torch.tensor(g.rho, device="cuda")
        bh.build_moments(rho)
        _cache[name] = (g, bh, rho, OracleTree(g))
    return _cache[name]


def _group_of_cell(nleaf):
    """canonical group id of every canonical cell, [nleaf, 8, 8, 8]"""
    k, j, i = np.meshgrid(np.arange(8), np.arange(8), np.arange(8), indexing="ij")
    m = np.zeros_like(i)
    for b in range(3):
        m |= ((i >> b) & 1) << (3 * b)
        m |= ((j >> b) & 1) << (3 * b + 1)
        m |= ((k >> b) & 1) << (3 * b + 2)
    return np.arange(nleaf)[:, None, None, None] * 8 + (m // 64)[None]


def _scale(ref):
    n = np.linalg.norm(ref, axis=-1)
    return np.maximum(n, 0.1 * np.sqrt((n * n).mean()))


@pytest.mark.parametrize("name", list(GRIDS))
@pytest.mark.parametrize("precision", [B.BH_FP64, B.BH_FP32])
@pytest.mark.parametrize("theta", [0.3, 0.7, 1.0])
def test_accel_matches_oracle(name, precision, theta):
    g, bh, rho, t = setup(name)
    ng = bh.info["n_groups"]
    acc = torch.full(g.rho.shape + (3,), float("nan"), dtype=torch.float64, device="cuda")
    phi = torch.empty_like(rho)
    counts = torch.zeros((ng, 2), dtype=torch.int32, device="cuda")
    B.bh_walk_accel(bh.ctx, bh.grid, bh.m, theta, None, precision, 1.0, phi, acc, counts)
    bh.check()
    ow = t.walk(64, theta, tau=TAU[precision])
    ref = t.accel()
    ref_phi = t.potential()
    clean_group = ow["marginal"] == 0
    c = counts.cpu().numpy()
    assert np.array_equal(c[clean_group, 0], ow["n_far"][clean_group])
    assert np.array_equal(c[clean_group, 1], ow["n_near"][clean_group])
    clean = clean_group[_group_of_cell(g.nleaf)]
    a = acc.cpu().numpy()
    err = np.linalg.norm(a - ref, axis=-1) / _scale(ref)
    assert np.all(err[clean] <= TOL[precision]), err[clean].max()
    p = phi.cpu().numpy()
    assert np.all(np.abs(p - ref_phi)[clean] <= TOL[precision] * np.abs(ref_phi)[clean])
    # accelerations only: the potential output may be left out
    acc2 = torch.empty_like(acc)
    B.bh_walk_accel(bh.ctx, bh.grid, bh.m, theta, None, precision, 1.0, None, acc2, None)
    assert torch.equal(acc, acc2)


@pytest.mark.parametrize("name", ["random_amr", "maclaurin_l1"])
def test_direct_accel_kernel(name):
    g, bh, rho, t = setup(name)
    rng = np.random.default_rng(4)
    tg = np.sort(rng.choice(g.ncells, 300, replace=False)).astype(np.int64)
    out = torch.empty((tg.size, 3), dtype=torch.float64, device="cuda")
    B.bh_direct_accel(bh.ctx, bh.grid, bh.m, torch.tensor(tg, device="cuda"), 1.0, out)
    ref = t.direct_accel(tg)
    err = np.linalg.norm(out.cpu().numpy() - ref, axis=1) / np.linalg.norm(ref, axis=1)
    assert err.max() <= 1e-12


def test_small_theta_is_direct_accel():
    g, bh, rho, t = setup("random_amr")
    acc = torch.empty(g.rho.shape + (3,), dtype=torch.float64, device="cuda")
    B.bh_walk_accel(bh.ctx, bh.grid, bh.m, 1e-4, None, B.BH_FP64, 1.0, None, acc, None)
    tg = torch.arange(g.ncells, dtype=torch.int64, device="cuda")
    d = torch.empty((g.ncells, 3), dtype=torch.float64, device="cuda")
    B.bh_direct_accel(bh.ctx, bh.grid, bh.m, tg, 1.0, d)
    ref = d.cpu().numpy()
    err = np.linalg.norm(acc.reshape(-1, 3).cpu().numpy() - ref, axis=1) / _scale(ref)
    assert err.max() <= 1e-11


def test_accel_invalid_arguments():
    g, bh, rho, t = setup("single_block")
    acc = torch.empty(g.rho.shape + (3,), dtype=torch.float64, device="cuda")
    with pytest.raises(B.BHError):
        B.bh_walk_accel(bh.ctx, bh.grid, bh.m, 1.5, None, B.BH_FP32, 1.0, None, acc)
    with pytest.raises(B.BHError):
        B.bh_walk_accel(bh.ctx, bh.grid, bh.m, 0.5, None, 7, 1.0, None, acc)
