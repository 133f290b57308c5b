"""FP64 oracle of the per-group features of the learned opening angle
(test infrastructure only), written from the definitions:

  0 log2(group cells)                     1 log(M_group / M_root)
  2 log(group edge / box)                 3 AMR level of the leaf block
  4 log(max / mean cell mass in group)    5,6 log(delta/l + 1e-6), log(|Q|_F/(M l^2) + 1e-6) of the group node
  7,8 the same for the leaf block         9,10 the same for the leaf block's parent node
  11 log(mean group density / mean density of the leaf block)

Node moments come from the oracle's own tree (brute force per node).
"""
import numpy as np

from .oracle import make_key


def _morton_decode(m):
    m = np.asarray(m)
    i = sum(((m >> (3 * p)) & 1) << p for p in range(3))
    j = sum(((m >> (3 * p + 1)) & 1) << p for p in range(3))
    k = sum(((m >> (3 * p + 2)) & 1) << p for p in range(3))
    return i, j, k


def group_features(tree, grid, group_cells=64):
    assert group_cells == 64
    mo = tree.moments()
    order = np.argsort(mo["key"])
    skeys = mo["key"][order]

    def idx(keys):
        pos = np.searchsorted(skeys, keys)
        out = order[pos]
        assert np.array_equal(mo["key"][out], keys)
        return out

    _, _, _, m = tree.cells()
    vlev = int(round(np.log2(grid.nbase)))
    lb = grid.leaf_blocks
    nleaf = len(lb)
    level = grid.level[lb].astype(np.int64)
    edge = grid.box_size / (grid.nbase * 2.0 ** level)
    corner = np.rint((grid.lo[lb] - grid.box_lo) / edge[:, None]).astype(np.int64)
    depth = vlev + level
    blk = idx(make_key(depth.astype(np.uint64), corner[:, 0].astype(np.uint64), corner[:, 1].astype(np.uint64),
                       corner[:, 2].astype(np.uint64)))
    pdepth = np.maximum(depth - 1, 0)
    pc = np.where(depth[:, None] > 0, corner >> 1, corner)
    par = idx(make_key(pdepth.astype(np.uint64), pc[:, 0].astype(np.uint64), pc[:, 1].astype(np.uint64),
                       pc[:, 2].astype(np.uint64)))
    root = idx(np.array([make_key(0, 0, 0, 0)], np.uint64))[0]
    F = np.zeros((nleaf * 8, 12))
    h = edge / 8
    for sub in range(8):
        oc = 2 * corner + np.array([sub & 1, (sub >> 1) & 1, (sub >> 2) & 1])
        grp = idx(make_key((depth + 1).astype(np.uint64), oc[:, 0].astype(np.uint64), oc[:, 1].astype(np.uint64),
                           oc[:, 2].astype(np.uint64)))
        i, j, k = _morton_decode(sub * 64 + np.arange(64))
        cid = np.arange(nleaf)[:, None] * 512 + (k * 64 + j * 8 + i)[None, :]
        cm = m[cid]
        rows = np.arange(nleaf) * 8 + sub
        Mg = mo["M"][grp]
        Mb = mo["M"][blk]
        Mr = mo["M"][root]
        F[rows, 0] = 6.0
        F[rows, 1] = np.log(np.maximum(Mg / Mr if Mr > 0 else 0.0 * Mg, 1e-30))
        F[rows, 2] = np.log(4 * h / grid.box_size)
        F[rows, 3] = level
        mean = cm.mean(1)
        F[rows, 4] = np.where(mean > 0, np.log(np.where(mean > 0, cm.max(1) / np.where(mean > 0, mean, 1), 1)), 0.0)
        for a, node in enumerate((grp, blk, par)):
            M = mo["M"][node]
            Q = mo["Q"][node]
            l = mo["edge"][node]
            qf = np.sqrt(Q[:, 0] ** 2 + Q[:, 1] ** 2 + Q[:, 2] ** 2 + 2 * (Q[:, 3] ** 2 + Q[:, 4] ** 2 + Q[:, 5] ** 2))
            F[rows, 5 + 2 * a] = np.log(mo["delta"][node] / l + 1e-6)
            F[rows, 6 + 2 * a] = np.log(np.where(M > 0, qf / np.where(M > 0, M * l * l, 1), 0.0) + 1e-6)
        F[rows, 11] = np.where(Mb > 0, np.log(np.maximum(8 * Mg / np.where(Mb > 0, Mb, 1), 1e-30)), 0.0)
    return F
