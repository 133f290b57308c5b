"""CPU-side checks of the library: it loads, exports every symbol that
include/bh.h declares, and its host topology builder agrees with the oracle's
independent tree (same node set by key) and rejects malformed grids.
No compute call is made here (no GPU)."""
import os
import re

import numpy as np
import pytest

from amr_inputs import maclaurin_spheroid, random_amr, single_block, uniform_sphere
from oracle import OracleTree

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
B = pytest.importorskip("paper_1509_07370_amd.binding")


def _declared():
    src = open(os.path.join(ROOT, "include", "bh.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(bh_[a-z_0-9]+)\s*\(", src)))


def test_every_declared_symbol_is_exported():
    names = _declared()
    assert len(names) >= 19
    for n in names:
        assert hasattr(B._lib, n), n
        assert n in B.EXPORTED, n


@pytest.fixture(scope="module")
def hctx():
    c = B.bh_ctx_create(-1)
    yield c
    B.bh_ctx_destroy(c)


@pytest.mark.parametrize("make", [single_block, lambda: random_amr(4, nbase=2, max_level=3, p_refine=0.3),
                                  lambda: uniform_sphere(), lambda: maclaurin_spheroid(max_level=1)])
def test_topology_matches_oracle_tree(hctx, make):
    g = make()
    h = B.bh_grid_create_from(hctx, g)
    try:
        info = B.bh_grid_info(h)
        keys = B.bh_grid_node_keys(h)
        t = OracleTree(g)
        ok = t.node_info()["key"]
        assert info["n_nodes"] == t.nnodes
        assert info["n_cells"] == g.ncells
        assert info["n_groups"] == g.ncells // 64
        assert np.array_equal(np.sort(keys), np.sort(ok))
        assert len(np.unique(keys)) == len(keys)
    finally:
        B.bh_grid_destroy(h)


def test_block_list_order_does_not_matter(hctx):
    g = random_amr(9, nbase=2, max_level=2, p_refine=0.4)
    perm = np.random.default_rng(0).permutation(g.nblocks)
    inv = np.empty_like(perm)
    inv[perm] = np.arange(g.nblocks)
    child = np.where(g.child[perm] >= 0, inv[np.maximum(g.child[perm], 0)], -1)
    parent = np.where(g.parent[perm] >= 0, inv[np.maximum(g.parent[perm], 0)], -1)
    h1 = B.bh_grid_create_from(hctx, g)
    h2 = B.bh_grid_create(hctx, g.level[perm], g.lo[perm], parent, child, g.is_leaf[perm], g.box_lo, g.box_size)
    try:
        assert np.array_equal(np.sort(B.bh_grid_node_keys(h1)), np.sort(B.bh_grid_node_keys(h2)))
    finally:
        B.bh_grid_destroy(h1)
        B.bh_grid_destroy(h2)


def _expect_einval(hctx, level, lo, parent, child, is_leaf, box_lo=(0, 0, 0), box=1.0, gc=64, nb=8, match=""):
    with pytest.raises(B.BHError) as ei:
        B.bh_grid_create(hctx, level, lo, parent, child, is_leaf, box_lo, box, gc, nb)
    assert ei.value.code == B.BH_EINVAL
    assert match in str(ei.value)


def test_malformed_grids_are_rejected(hctx):
    g = random_amr(4, nbase=2, max_level=2, p_refine=0.4)
    a = dict(level=g.level.copy(), lo=g.lo.copy(), parent=g.parent.copy(), child=g.child.copy(),
             is_leaf=g.is_leaf.copy())
    _expect_einval(hctx, **a, nb=16, match="nb must be 8")
    _expect_einval(hctx, **a, gc=48, match="group_cells")
    _expect_einval(hctx, **a, gc=1024, match="group_cells")
    b = {k: v.copy() for k, v in a.items()}
    b["lo"][3, 0] += 1e-3
    _expect_einval(hctx, **b, match="lattice")
    refined = int(np.nonzero(g.is_leaf == 0)[0][0])
    b = {k: v.copy() for k, v in a.items()}
    b["child"][refined, 2] = -1
    _expect_einval(hctx, **b, match="lacks child")
    b = {k: v.copy() for k, v in a.items()}
    c = int(g.child[refined, 0])
    b["parent"][c] = -1
    _expect_einval(hctx, **b)
    b = {k: v.copy() for k, v in a.items()}
    b["level"] = b["level"][1:]
    b["lo"] = b["lo"][1:]
    b["parent"] = b["parent"][1:]
    b["child"] = b["child"][1:]
    b["is_leaf"] = b["is_leaf"][1:]
    _expect_einval(hctx, **b)
    _expect_einval(hctx, **a, box=-1.0, match="box_size")


def test_host_context_refuses_gpu_work(hctx):
    g = single_block()
    h = B.bh_grid_create_from(hctx, g)
    try:
        m = B.ctypes.c_void_p()
        rc = B._lib.bh_build_moments(hctx, h, B.ctypes.c_void_p(1), B.ctypes.byref(m))
        assert rc == B.BH_ESTATE
        assert "host-only" in B.bh_last_error(hctx)
    finally:
        B.bh_grid_destroy(h)
