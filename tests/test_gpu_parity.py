"""GPU path vs the CPU oracle, through the C ABI.

* moments: every node, fp64, against the oracle's brute-force moments;
* walk: interaction lists identical to the oracle's per group, except groups
  holding a decision the oracle flags as marginal (|d^2 - s^2| <= tau s^2);
* potential: the oracle re-evaluates the GPU's own lists in fp64 (list
  replay) -- fp64 path within 1e-12, fp32 path within 1e-5 per cell -- and the
  fp64 path also matches the oracle's own walk + sum within 1e-12;
* direct sum: fp64 within 1e-12 of the oracle on sampled targets;
* edge cases: one-block grid, zero-mass blocks, all-zero density, per-group
  theta, invalid inputs.
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
        t = OracleTree(g)
        t.moments()
        _cache[name] = (g, bh, rho, t, bh.node_keys())
    return _cache[name]


def _by_key(keys_a, keys_b):
    """index into b for every key of a"""
    order = np.argsort(keys_b)
    pos = np.searchsorted(keys_b, keys_a, sorter=order)
    idx = order[pos]
    assert np.array_equal(keys_b[idx], keys_a)
    return idx


@pytest.mark.parametrize("name", list(GRIDS))
def test_moments_parity(name):
    g, bh, rho, t, keys = setup(name)
    gm = bh.moments_host()
    om = t.moments()
    idx = _by_key(keys, om["key"])
    M, X, Q, d = om["M"][idx], om["X"][idx], om["Q"][idx], om["delta"][idx]
    l = om["edge"][idx]
    assert np.all(np.abs(gm["M"] - M) <= 1e-13 * M)
    assert np.max(np.abs(gm["X"] - X)) <= 4e-15 * g.box_size
    assert np.all(np.abs(gm["Q"] - Q) <= 1e-13 * (M * l * l)[:, None] + 1e-300)
    assert np.max(np.abs(gm["delta"] - d)) <= 4e-15 * g.box_size


def _check_moments(g, gm, om, keys):
    idx = _by_key(keys, om["key"])
    M, X, Q, d = om["M"][idx], om["X"][idx], om["Q"][idx], om["delta"][idx]
    l = om["edge"][idx]
    assert np.all(np.abs(gm["M"] - M) <= 1e-13 * M)
    assert np.max(np.abs(gm["X"] - X)) <= 4e-15 * g.box_size
    assert np.all(np.abs(gm["Q"] - Q) <= 1e-13 * (M * l * l)[:, None] + 1e-300)
    assert np.max(np.abs(gm["delta"] - d)) <= 4e-15 * g.box_size


@pytest.mark.parametrize("seed,nbase,max_level", [(33, 2, 4), (34, 1, 5), (35, 4, 2)])
def test_repeated_upward_passes(seed, nbase, max_level):
    """Upward passes in a row, with densities that change (zero blocks
    included), on deep and shallow trees: each must give the oracle's moments
    (nothing may carry over between calls)."""
    g = random_amr(seed, nbase=nbase, max_level=max_level, p_refine=0.35, zero_fraction=0.1)
    bh = BarnesHut(g)
    keys = bh.node_keys()
    t = OracleTree(g)
    rng = np.random.default_rng(seed)
    for rep in range(4):
        rho_h = g.rho.copy() if rep == 0 else g.rho * rng.uniform(0.5, 2.0, size=g.rho.shape)
        if rep == 3:
            rho_h[::3] = 0.0
        bh.build_moments(torch.tensor(rho_h, device="cuda"))
        bh.check()
        t.set_density(rho_h)
        _check_moments(g, bh.moments_host(), t.moments(), keys)
    bh.close()


def _gpu_lists_as_keys(bh, keys):
    L = bh.lists_host()
    return L["far_off"], keys[L["far_node"]], L["near_off"], keys[L["near_node"]]


def _compare_lists(t, bh, keys, theta, precision):
    ow = t.walk(64, theta, tau=TAU[precision])
    fo, fk, no, nk = _gpu_lists_as_keys(bh, keys)
    ng = len(fo) - 1
    differ = []
    for q in range(ng):
        a = np.sort(fk[fo[q]:fo[q + 1]])
        b = np.sort(ow["far_keys"][ow["far_off"][q]:ow["far_off"][q + 1]])
        c = np.sort(nk[no[q]:no[q + 1]])
        d = np.sort(ow["near_keys"][ow["near_off"][q]:ow["near_off"][q + 1]])
        if not (np.array_equal(a, b) and np.array_equal(c, d)):
            differ.append(q)
    differ = np.array(differ, dtype=np.int64)
    # every differing group holds a marginal decision, and they are rare
    assert np.all(ow["marginal"][differ] > 0) if differ.size else True
    assert differ.size <= max(1, ng // 1000)
    return ow, (fo, fk, no, nk)


@pytest.mark.parametrize("name", list(GRIDS))
@pytest.mark.parametrize("precision", [B.BH_FP64, B.BH_FP32])
@pytest.mark.parametrize("theta", [0.3, 0.7])
def test_walk_decision_parity(name, precision, theta):
    g, bh, rho, t, keys = setup(name)
    bh.walk(theta, None, precision)
    _compare_lists(t, bh, keys, theta, precision)


@pytest.mark.parametrize("name", list(GRIDS))
@pytest.mark.parametrize("theta", [0.3, 0.7])
def test_potential_fp64_parity(name, theta):
    g, bh, rho, t, keys = setup(name)
    bh.walk(theta, None, B.BH_FP64)
    phi = torch.empty_like(rho)
    bh.potential(phi, 1.0, B.BH_FP64)
    got = phi.cpu().numpy()
    ow, (fo, fk, no, nk) = _compare_lists(t, bh, keys, theta, B.BH_FP64)
    replay = t.potential_lists(64, fo, fk, no, nk)
    assert np.max(np.abs(got - replay) / np.abs(replay)) <= 1e-12
    own = t.potential()  # the oracle's own walk (differs only in marginal groups)
    ok = np.repeat(ow["marginal"] == 0, 64).reshape(got.shape[0], -1)
    rel = np.abs(got - own) / np.abs(own)
    assert np.max(rel.reshape(got.shape[0], -1)[ok]) <= 1e-12


@pytest.mark.parametrize("name", list(GRIDS))
@pytest.mark.parametrize("theta", [0.3, 0.7, 1.0])
def test_potential_fp32_parity(name, theta):
    g, bh, rho, t, keys = setup(name)
    bh.walk(theta, None, B.BH_FP32)
    phi = torch.empty_like(rho)
    bh.potential(phi, 1.0, B.BH_FP32)
    got = phi.cpu().numpy()
    L = bh.lists_host()
    replay = t.potential_lists(64, L["far_off"], keys[L["far_node"]], L["near_off"], keys[L["near_node"]])
    assert np.max(np.abs(got - replay) / np.abs(replay)) <= 1e-5


@pytest.mark.parametrize("name", ["random_amr", "maclaurin_l1"])
def test_direct_parity(name):
    g, bh, rho, t, keys = setup(name)
    rng = np.random.default_rng(5)
    tg = np.sort(rng.choice(g.ncells, 300, replace=False)).astype(np.int64)
    tg[0] = 0
    tg[-1] = g.ncells - 1
    got = bh.direct(torch.tensor(tg, device="cuda")).cpu().numpy()
    ref = t.direct(tg)
    assert np.max(np.abs(got - ref) / np.abs(ref)) <= 1e-12


def test_per_group_theta_parity():
    g, bh, rho, t, keys = setup("random_amr")
    ng = bh.info["n_groups"]
    th = np.random.default_rng(2).uniform(0.25, 1.0, ng).astype(np.float32)
    bh.walk(0.5, torch.tensor(th, device="cuda"), B.BH_FP64)
    phi = torch.empty_like(rho)
    bh.potential(phi, 1.0, B.BH_FP64)
    ow = t.walk(64, th.astype(np.float64), tau=1e-12)
    own = t.potential()
    got = phi.cpu().numpy()
    ok = np.repeat(ow["marginal"] == 0, 64).reshape(got.shape[0], -1)
    rel = (np.abs(got - own) / np.abs(own)).reshape(got.shape[0], -1)
    assert np.max(rel[ok]) <= 1e-12


def test_method_error_vs_direct_fp32():
    g, bh, rho, t, keys = setup("sphere")
    bh.walk(0.5, None, B.BH_FP32)
    phi = torch.empty_like(rho)
    bh.potential(phi, 1.0, B.BH_FP32)
    d = bh.direct(torch.arange(g.ncells, device="cuda", dtype=torch.int64))
    # direct targets are canonical ids = flat index of the caller layout
    rel = ((phi.reshape(-1) - d) / d).abs()
    assert float(torch.sqrt((rel ** 2).mean())) <= 1e-3


def test_zero_density_gives_zero_potential():
    g = random_amr(3, nbase=2, max_level=1, p_refine=0.5)
    bh = BarnesHut(g)
    rho = torch.zeros(g.rho.shape, dtype=torch.float64, device="cuda")
    for prec in (B.BH_FP64, B.BH_FP32):
        phi = bh.solve(rho, 0.5, precision=prec)
        assert float(phi.abs().max()) == 0.0
        nf, nn = B.bh_lists_info(bh.lists)
        assert nf == 0 and nn == 0
    # the fused walk, the learned-theta step, accelerations and the periodic box: zero as well, no node visited
    import os
    from paper_1509_07370_amd import learned_theta as LT
    ng = bh.info["n_groups"]
    counts = torch.full((ng, 2), -1, dtype=torch.int32, device="cuda")
    phi = torch.full_like(rho, float("nan"))
    acc = torch.full(tuple(rho.shape) + (3,), float("nan"), dtype=torch.float64, device="cuda")
    net = LT.ThetaNet.load(bh.ctx, os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                                                "paper_1509_07370_amd", "data", "theta_mlp_1e-3.npz"))
    table = B.bh_ewald_create(bh.ctx, g.box_size, 9)
    bh.build_moments(rho)
    for prec in (B.BH_FP64, B.BH_FP32):
        runs = [lambda: B.bh_walk_potential(bh.ctx, bh.grid, bh.m, 0.5, None, prec, 1.0, phi, counts),
                lambda: B.bh_learned_walk_potential(bh.ctx, bh.grid, bh.m, net.h, net.shift, prec, 1.0, phi, None,
                                                    counts),
                lambda: B.bh_walk_accel(bh.ctx, bh.grid, bh.m, 0.5, None, prec, 1.0, phi, acc, counts),
                lambda: B.bh_walk_potential_periodic(bh.ctx, bh.grid, bh.m, table, 0.5, None, prec, 1.0, phi, counts)]
        for run in runs:
            phi.fill_(float("nan"))
            counts.fill_(-1)
            run()
            bh.check()
            assert float(phi.abs().max()) == 0.0
            assert int(counts.abs().max()) == 0
        assert float(acc.abs().max()) == 0.0
    B.bh_ewald_destroy(table)
    net.close()
    bh.close()


def test_invalid_inputs_raise():
    g = single_block()
    bh = BarnesHut(g)
    rho = torch.tensor(g.rho, device="cuda")
    bh.build_moments(rho)
    for bad_theta in (0.0, -0.5, 1.5, float("nan")):
        with pytest.raises(B.BHError) as ei:
            bh.walk(bad_theta, None, B.BH_FP32)
        assert ei.value.code == B.BH_EINVAL
    with pytest.raises(B.BHError):
        bh.walk(0.5, None, 7)
    bad = rho.clone()
    bad[0, 1, 2, 3] = -1.0
    bh.build_moments(bad)
    with pytest.raises(B.BHError) as ei:
        B.bh_moments_check(bh.ctx, bh.m)
    assert ei.value.code == B.BH_EINVAL
    with pytest.raises(B.BHError) as ei:
        bh.walk(0.5, None, B.BH_FP32)
    assert ei.value.code == B.BH_EINVAL
    bad[0, 1, 2, 3] = float("nan")
    bh.build_moments(bad)
    with pytest.raises(B.BHError):
        bh.walk(0.5, None, B.BH_FP32)
    bh.build_moments(rho)
    bh.walk(0.5, None, B.BH_FP32)  # recovers
    with pytest.raises(TypeError):
        bh.build_moments(rho.float())
    bh.close()


@pytest.mark.parametrize("name", list(GRIDS))
@pytest.mark.parametrize("precision", [B.BH_FP64, B.BH_FP32])
@pytest.mark.parametrize("theta", [0.3, 0.7])
def test_fused_walk_potential_equals_list_path(name, precision, theta):
    """bh_walk_potential forms the same tiles in the same order: identical bits."""
    g, bh, rho, t, keys = setup(name)
    bh.walk(theta, None, precision)
    ref = torch.empty_like(rho)
    bh.potential(ref, 1.0, precision)
    got = torch.empty_like(rho)
    counts = torch.zeros((bh.info["n_groups"], 2), dtype=torch.int32, device="cuda")
    B.bh_walk_potential(bh.ctx, bh.grid, bh.m, theta, None, precision, 1.0, got, counts)
    bh.check()
    assert torch.equal(got, ref)
    L = bh.lists_host()
    c = counts.cpu().numpy()
    assert np.array_equal(c[:, 0], np.diff(L["far_off"]))
    assert np.array_equal(c[:, 1], np.diff(L["near_off"]))


def test_fused_per_group_theta_and_invalid_density():
    g, bh, rho, t, keys = setup("random_amr")
    ng = bh.info["n_groups"]
    th = torch.tensor(np.random.default_rng(4).uniform(0.2, 1.0, ng).astype(np.float32), device="cuda")
    bh.walk(0.5, th, B.BH_FP32)
    ref = torch.empty_like(rho)
    bh.potential(ref, 2.5, B.BH_FP32)
    got = torch.empty_like(rho)
    B.bh_walk_potential(bh.ctx, bh.grid, bh.m, 0.5, th, B.BH_FP32, 2.5, got, None)
    assert torch.equal(got, ref)
    bad = rho.clone()
    bad[1, 0, 0, 0] = -2.0
    bh.build_moments(bad)
    B.bh_walk_potential(bh.ctx, bh.grid, bh.m, 0.5, None, B.BH_FP32, 1.0, got, None)
    with pytest.raises(B.BHError) as ei:
        bh.check()
    assert ei.value.code == B.BH_EINVAL
    bh.build_moments(rho)
    B.bh_walk_potential(bh.ctx, bh.grid, bh.m, 0.5, None, B.BH_FP32, 1.0, got, None)
    bh.check()
