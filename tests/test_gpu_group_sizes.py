"""Group size as a parameter: groups of 32, 64, 128, 256 and 512 cells against
the oracle's walk with the same partition (O4: aligned Morton runs of
group_cells cells; the paper's own group is a 32-cell warp), through the C ABI.

* list path: interaction lists identical to the oracle's outside groups with
  a marginal decision; potentials by list replay (fp64 1e-12, fp32 1e-5) and
  against the oracle's own walk and sum (fp64 1e-12);
* fused path: groups of 64 or more cells give the list path's bits (each
  wavefront of a multi-wavefront group walks the same tree); 32-cell groups
  (two per wavefront, lists kept apart by masks) match the oracle's walk and
  sum (fp64 1e-12, fp32 1e-5) with the oracle's counts;
* per-group theta arrays, the paper's cube test with the monopole far field,
  accelerations and the no-allocation entry point at 32 and 128 cells;
* the periodic walk at 32, 128 and 512 cells (on the random grid the
  finest level sums the Ewald term's smooth part through the octant's cubic,
  the next through bottom-node cubics, the coarser pair by pair; 32-cell
  groups always pair by pair) against the oracle's O10 with the same
  partition, within each group's derived bound;
* bad group sizes, and calls that need 64-cell groups, are refused.
"""
import numpy as np
import pytest

from amr_inputs import maclaurin_spheroid, random_amr

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from oracle import OracleTree
from oracle.oracle import fp32_band_for  # noqa: E402
from periodic_bounds import (DELTA, EPS_FP32_ROWS, EPS_FP64_ROWS, N_TABLE, local_axis, local_reach,  # noqa: E402
                             storage_terms, walk_tolerance)
from paper_1509_07370_amd import binding as B  # noqa: E402
from paper_1509_07370_amd.solver import BarnesHut  # noqa: E402

SIZES = [32, 64, 128, 256, 512]
# fp32: the band derived from fp32 rounding (every test grid lies in the unit box)
TAU = {B.BH_FP64: 1e-12, B.BH_FP32: fp32_band_for(1.0)}
GRIDS = {
    "random_amr": lambda: random_amr(21, nbase=2, max_level=3, p_refine=0.3, zero_fraction=0.1),
    "maclaurin_l1": lambda: maclaurin_spheroid(max_level=1),
}
_grids, _oracles, _solvers = {}, {}, {}


def setup(name, G):
    if name not in _grids:
        _grids[name] = GRIDS[name]()
        t = OracleTree(_grids[name])
        t.moments()
        _oracles[name] = t
    g = _grids[name]
    if (name, G) not in _solvers:
        bh = BarnesHut(g, group_cells=G)
        rho = torch.tensor(g.rho, device="cuda")
        bh.build_moments(rho)
        _solvers[(name, G)] = (bh, rho, bh.node_keys())
    bh, rho, keys = _solvers[(name, G)]
    return g, bh, rho, _oracles[name], keys


def group_cells_canonical(G, ng_leaf_groups, groups):
    """canonical cell ids of canonical groups (aligned Morton runs of G cells)"""
    out = []
    per = 512 // G
    for q in groups:
        m = np.arange(G) + (q % per) * G
        i = sum(((m >> (3 * b)) & 1) << b for b in range(3))
        j = sum(((m >> (3 * b + 1)) & 1) << b for b in range(3))
        k = sum(((m >> (3 * b + 2)) & 1) << b for b in range(3))
        out.append((q // per) * 512 + k * 64 + j * 8 + i)
    return np.array(out)


def _lists(bh, keys):
    L = bh.lists_host()
    return L["far_off"], keys[L["far_node"]], L["near_off"], keys[L["near_node"]]


def _compare(ow, fo, fk, no, nk):
    ng = len(fo) - 1
    differ = [q for q in range(ng) if not (
        np.array_equal(np.sort(fk[fo[q]:fo[q + 1]]), np.sort(ow["far_keys"][ow["far_off"][q]:ow["far_off"][q + 1]]))
        and np.array_equal(np.sort(nk[no[q]:no[q + 1]]),
                           np.sort(ow["near_keys"][ow["near_off"][q]:ow["near_off"][q + 1]])))]
    differ = np.array(differ, dtype=np.int64)
    assert (np.all(ow["marginal"][differ] > 0) if differ.size else True), differ
    # fp32 rounding may flip a decision within the marginal band; larger groups test more cells per node, so
    # such groups are a little more frequent than with 64 cells (two of 1488 128-cell groups on the random grid)
    assert differ.size <= max(2, ng // 200)


@pytest.mark.parametrize("name", list(GRIDS))
@pytest.mark.parametrize("G", SIZES)
@pytest.mark.parametrize("precision", [B.BH_FP64, B.BH_FP32])
def test_list_path_parity(name, G, precision):
    g, bh, rho, t, keys = setup(name, G)
    assert bh.info["group_cells"] == G and bh.info["n_groups"] == g.ncells // G
    theta = 0.6
    bh.walk(theta, None, precision)
    ow = t.walk(G, theta, tau=TAU[precision])
    fo, fk, no, nk = _lists(bh, keys)
    _compare(ow, fo, fk, no, nk)
    phi = torch.empty_like(rho)
    bh.potential(phi, 1.0, precision)
    got = phi.cpu().numpy()
    replay = t.potential_lists(G, fo, fk, no, nk)
    tol = 1e-12 if precision == B.BH_FP64 else 1e-5
    assert np.max(np.abs(got - replay) / np.abs(replay)) <= tol
    if precision == B.BH_FP64:
        own = t.potential()
        ok = np.zeros(g.ncells, bool)
        clean = np.nonzero(ow["marginal"] == 0)[0]
        ok[group_cells_canonical(G, None, clean).ravel()] = True
        rel = (np.abs(got - own) / np.abs(own)).reshape(-1)
        assert np.max(rel[ok]) <= 1e-12


@pytest.mark.parametrize("name", list(GRIDS))
@pytest.mark.parametrize("G", SIZES)
@pytest.mark.parametrize("precision", [B.BH_FP64, B.BH_FP32])
def test_fused_path(name, G, precision):
    g, bh, rho, t, keys = setup(name, G)
    theta = 0.7
    ng = bh.info["n_groups"]
    counts = torch.full((ng, 2), -1, dtype=torch.int32, device="cuda")
    phi = torch.full_like(rho, float("nan"))
    bh.build_moments(rho)
    B.bh_walk_potential(bh.ctx, bh.grid, bh.m, theta, None, precision, 1.0, phi, counts)
    bh.check()
    ow = t.walk(G, theta, tau=TAU[B.BH_FP32])
    c = counts.cpu().numpy()
    clean = ow["marginal"] == 0
    assert np.array_equal(c[clean, 0], ow["n_far"][clean]) and np.array_equal(c[clean, 1], ow["n_near"][clean])
    if G >= 64:
        bh.walk(theta, None, precision)
        ref = torch.empty_like(rho)
        bh.potential(ref, 1.0, precision)
        assert torch.equal(phi, ref)
    own = t.potential().reshape(-1)
    got = phi.cpu().numpy().reshape(-1)
    ok = np.zeros(g.ncells, bool)
    ok[group_cells_canonical(G, None, np.nonzero(clean)[0]).ravel()] = True
    tol = 1e-12 if precision == B.BH_FP64 else 1e-5
    assert np.max(np.abs(got - own)[ok] / np.abs(own)[ok]) <= tol


@pytest.mark.parametrize("G", [32, 128])
def test_per_group_theta(G):
    g, bh, rho, t, keys = setup("random_amr", G)
    ng = bh.info["n_groups"]
    th = np.random.default_rng(G).uniform(0.3, 1.0, ng).astype(np.float32)
    phi = torch.empty_like(rho)
    bh.build_moments(rho)
    B.bh_walk_potential(bh.ctx, bh.grid, bh.m, 0.5, torch.tensor(th, device="cuda"), B.BH_FP64, 1.0, phi, None)
    ow = t.walk(G, th.astype(np.float64), tau=1e-12)
    own = t.potential().reshape(-1)
    ok = np.zeros(g.ncells, bool)
    ok[group_cells_canonical(G, None, np.nonzero(ow["marginal"] == 0)[0]).ravel()] = True
    got = phi.cpu().numpy().reshape(-1)
    assert np.max(np.abs(got - own)[ok] / np.abs(own)[ok]) <= 1e-12


@pytest.mark.parametrize("G", [32, 128])
@pytest.mark.parametrize("precision", [B.BH_FP64, B.BH_FP32])
def test_paper_cube_test_and_monopole(G, precision):
    """The paper's configuration at its own group size (32 cells): the cube test and the monopole far field."""
    g, bh, rho, t, keys = setup("maclaurin_l1", G)
    ng = bh.info["n_groups"]
    counts = torch.full((ng, 2), -1, dtype=torch.int32, device="cuda")
    phi = torch.empty_like(rho)
    bh.build_moments(rho)
    B.bh_walk_potential_ex(bh.ctx, bh.grid, bh.m, 0.5, None, precision, 1.0, phi, counts, mac=B.BH_MAC_GROUP_BOX,
                           order=0)
    bh.check()
    rng = np.random.default_rng(3)
    gs = np.unique(np.r_[0, ng - 1, rng.choice(ng, 40, replace=False)])
    ref, oc = t.solve_groups(gs, group_cells=G, theta=0.5, tau=TAU[B.BH_FP32], order=0, mac=1)
    cells = group_cells_canonical(G, None, gs)
    got = phi.cpu().numpy().reshape(-1)[cells]
    clean = oc[:, 3] == 0
    c = counts.cpu().numpy()[gs]
    assert np.array_equal(c[clean, 0], oc[clean, 1]) and np.array_equal(c[clean, 1], oc[clean, 2])
    tol = 1e-12 if precision == B.BH_FP64 else 1e-5
    assert np.max(np.abs(got[clean] - ref[clean]) / np.abs(ref[clean])) <= tol


@pytest.mark.parametrize("G", [32, 128])
def test_accelerations(G):
    g, bh, rho, t, keys = setup("random_amr", G)
    ng = bh.info["n_groups"]
    acc = torch.empty(tuple(rho.shape) + (3,), dtype=torch.float64, device="cuda")
    bh.build_moments(rho)
    B.bh_walk_accel(bh.ctx, bh.grid, bh.m, 0.6, None, B.BH_FP64, 1.0, None, acc, None)
    gs = np.unique(np.r_[0, ng - 1, np.random.default_rng(5).choice(ng, 30, replace=False)])
    ref, oc = t.solve_groups_accel(gs, group_cells=G, theta=0.6, tau=1e-12)
    cells = group_cells_canonical(G, None, gs)
    got = acc.cpu().numpy().reshape(-1, 3)[cells.ravel()].reshape(len(gs), G, 3)
    clean = oc[:, 3] == 0
    scale = np.maximum(np.linalg.norm(ref, axis=2), 0.1 * np.sqrt(np.mean(np.sum(ref ** 2, axis=2))))
    err = np.linalg.norm(got - ref, axis=2) / scale
    assert np.max(err[clean]) <= 1e-12


_periodic_oracle = {}


@pytest.mark.parametrize("G", [32, 128, 512])
@pytest.mark.parametrize("precision", [B.BH_FP64, B.BH_FP32])
def test_periodic(G, precision):
    g, bh, rho, t, keys = setup("random_amr", G)
    ng = bh.info["n_groups"]
    table = B.bh_ewald_create(bh.ctx, g.box_size, N_TABLE)
    phi = torch.full_like(rho, float("nan"))
    counts = torch.full((ng, 2), -1, dtype=torch.int32, device="cuda")
    bh.build_moments(rho)
    B.bh_walk_potential_periodic(bh.ctx, bh.grid, bh.m, table, 0.7, None, precision, 1.0, phi, counts)
    bh.check()
    per = 512 // G
    lv = np.asarray(g.level)[np.asarray(g.leaf_blocks)]
    hg_all = g.box_size / (g.nbase * 8 * 2.0 ** lv[np.arange(ng) // per])
    fp32 = precision == B.BH_FP32
    axis_all = np.array([local_axis(h, B.EWALD_LOCAL_BUDGET, g.box_size) if G >= 64 else 0.0 for h in hg_all])
    if G not in _periodic_oracle:  # a few random groups and one of each cell size, shared by both precisions
        rng = np.random.default_rng(G)
        sizes = [rng.choice(np.flatnonzero(hg_all == h)) for h in np.unique(hg_all)]
        gs = np.unique(np.concatenate([rng.choice(ng, 5, replace=False), sizes]))
        _periodic_oracle[G] = (gs,) + tuple(t.solve_groups_periodic(gs, group_cells=G, theta=0.7,
                                                                     tau=TAU[B.BH_FP32], with_qsum=True))
    gs, ref, oc, qs = _periodic_oracle[G]
    clean = oc[:, 3] == 0
    c = counts.cpu().numpy()[gs]
    assert clean.sum() >= 3
    assert np.array_equal(c[clean, 0], oc[clean, 1]) and np.array_equal(c[clean, 1], oc[clean, 2])
    got = phi.cpu().numpy().reshape(-1)[group_cells_canonical(G, None, gs).ravel()].reshape(len(gs), G)
    _, _, _, m = t.cells()
    exported = B.bh_ewald_export(bh.ctx, table, N_TABLE)
    eps = EPS_FP32_ROWS if fp32 else EPS_FP64_ROWS
    ax, hg = axis_all[gs], hg_all[gs]
    tol = np.array([walk_tolerance(m.sum(), qs[k], g.box_size, storage_terms(exported, g.box_size, eps, ax[k] * hg[k]),
                                   fp32, local_reach(hg[k], g.box_size, ax[k]) if ax[k] > 0 else DELTA)
                    for k in range(len(gs))])
    ratio = np.max(np.abs(got - ref), axis=1) / tol
    print("[periodic G=%d precision %d] %d groups, cubic placements %s, largest diff/tolerance %.2e"
          % (G, precision, clean.sum(), np.unique(ax[clean]).tolist(), ratio[clean].max()))
    assert np.all(ratio[clean] <= 1.0), ratio
    if G >= 64:
        assert len(np.unique(axis_all)) == 3  # octant, bottom node and pair by pair all occur on this grid
    B.bh_ewald_destroy(table)


@pytest.mark.parametrize("G", [32, 256])
def test_no_allocation_entry_point(G):
    g, bh, rho, t, keys = setup("random_amr", G)
    ng = bh.info["n_groups"]
    phi, ref = torch.empty_like(rho), torch.empty_like(rho)
    c1, c2 = (torch.zeros((ng, 2), dtype=torch.int32, device="cuda") for _ in range(2))
    B.bh_potential_static(bh.ctx, bh.grid, rho, 0.8, None, B.BH_FP32, 1.0, phi, c1, None)
    bh.build_moments(rho)
    B.bh_walk_potential(bh.ctx, bh.grid, bh.m, 0.8, None, B.BH_FP32, 1.0, ref, c2)
    torch.cuda.synchronize()
    assert torch.equal(phi, ref) and torch.equal(c1, c2)


def test_bad_group_sizes_and_restricted_calls():
    g = random_amr(5, nbase=2, max_level=1)
    ctx = B.bh_ctx_create(0)
    for G in (0, 16, 48, 1024):
        with pytest.raises(B.BHError) as ei:
            B.bh_grid_create_from(ctx, g, G)
        assert ei.value.code == B.BH_EINVAL
    B.bh_ctx_destroy(ctx)
    _, bh, rho, _, _ = setup("random_amr", 128)
    ng = bh.info["n_groups"]
    feat = torch.empty((ng, B.MLP_INPUTS), dtype=torch.float32, device="cuda")
    with pytest.raises(B.BHError) as ei:
        B.bh_group_features(bh.ctx, bh.grid, bh.m, feat)
    assert ei.value.code == B.BH_EINVAL
    with pytest.raises(B.BHError) as ei:
        B.bh_batch_create(bh.ctx, [bh.grid])
    assert ei.value.code == B.BH_EINVAL
