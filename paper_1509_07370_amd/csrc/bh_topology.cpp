// Host topology builder: AMR block list -> octree node arrays.
//
// The tree is the one of section 2 on an AMR mesh (the octree is the AMR
// block tree continued down to the cells): a root box, log2(nbase) virtual
// levels above the base blocks, the AMR blocks, and inside every leaf block
// 8 octant nodes (4^3 cells) and 64 bottom nodes (2^3 cells) whose children
// are the cells.  No insertion or locking (the paper's tree-building kernel,
// section 3.2.2) is needed: the AMR mesh already fixes the tree.
//
// Node ids are breadth-first, so the 8 children of every node are
// consecutive; leaf blocks (and therefore cells and groups) are numbered
// depth-first, i.e. in Morton order of space, so that consecutive groups are
// neighbours and walk similar parts of the tree.
#include <cmath>
#include <cstdio>
#include <algorithm>
#include <functional>
#include <unordered_map>

#include "bh_internal.h"

namespace bh {
namespace {

enum Kind : uint8_t { VIRTUAL, PARENT_BLOCK, LEAF_BLOCK, OCTANT, BOTTOM };

struct Desc {
    uint8_t kind;
    int depth;
    int64_t ix, iy, iz;
    int ref;  // block id (blocks), internal leaf (in-block nodes)
    int sub;  // octant (OCTANT) or 6-bit Morton index of the 2^3 sub-cube (BOTTOM)
};

uint64_t make_key(int depth, int64_t ix, int64_t iy, int64_t iz) {
    return ((uint64_t)depth << 57) | ((uint64_t)ix << 38) | ((uint64_t)iy << 19) | (uint64_t)iz;
}

std::string fmt(const char *f, long long a, long long b = 0, long long c = 0) {
    char buf[256];
    snprintf(buf, sizeof buf, f, a, b, c);
    return buf;
}

}  // namespace

std::string build_topology(Topology &t, int n, const int32_t *level, const double *lo, const int32_t *parent,
                           const int32_t *child, const uint8_t *is_leaf, const double box_lo[3], double box) {
    if (n <= 0) return "n_blocks must be positive";
    if (!(box > 0.0) || !std::isfinite(box)) return "box_size must be positive and finite";
    for (int d = 0; d < 3; d++)
        if (!std::isfinite(box_lo[d])) return "box_lo must be finite";
    int n0 = 0, maxlev = 0;
    for (int b = 0; b < n; b++) {
        if (level[b] < 0) return fmt("block %lld has a negative level", b);
        if (level[b] == 0) n0++;
        if (level[b] > maxlev) maxlev = level[b];
        if (is_leaf[b] > 1) return fmt("block %lld: is_leaf must be 0 or 1", b);
    }
    int nbase = 1;
    while ((int64_t)nbase * nbase * nbase < n0) nbase *= 2;
    if ((int64_t)nbase * nbase * nbase != n0)
        return fmt("%lld base (level-0) blocks do not form an nbase^3 lattice with nbase a power of two", n0);
    int vlev = 0;
    while ((1 << vlev) < nbase) vlev++;
    if (vlev + maxlev + 2 > kMaxDepth)
        return fmt("tree too deep: %lld virtual + %lld AMR levels (at most 16 in total)", vlev, maxlev);
    t.nbase = nbase;
    t.vlev = vlev;
    t.box = box;
    for (int d = 0; d < 3; d++) t.box_lo[d] = box_lo[d];
    t.nblocks = n;
    t.n_levels = maxlev + 1;

    // integer lattice position of every block
    std::vector<int64_t> pos((size_t)n * 3);
    std::unordered_map<uint64_t, int> where;
    where.reserve((size_t)n * 2);
    for (int b = 0; b < n; b++) {
        int64_t span = (int64_t)nbase << level[b];
        double e = box / (double)span;
        for (int d = 0; d < 3; d++) {
            double v = lo[3 * b + d];
            if (!std::isfinite(v)) return fmt("block %lld: lower corner not finite", b);
            double q = (v - box_lo[d]) / e;
            double r = std::nearbyint(q);
            if (std::fabs(q - r) > 1e-9 * (1.0 + std::fabs(q)) || r < 0 || r >= (double)span)
                return fmt("block %lld: lower corner is not on the level-%lld block lattice (axis %lld)", b,
                           level[b], d);
            pos[3 * b + d] = (int64_t)r;
        }
        uint64_t k = make_key(level[b], pos[3 * b], pos[3 * b + 1], pos[3 * b + 2]);
        if (!where.emplace(k, b).second) return fmt("blocks %lld and %lld occupy the same place", where[k], b);
    }
    for (int b = 0; b < n; b++) {
        if ((parent[b] < 0) != (level[b] == 0))
            return fmt("block %lld: parent must be -1 exactly for level-0 blocks", b);
        if (parent[b] >= n) return fmt("block %lld: parent index out of range", b);
        if (parent[b] >= 0) {
            int p = parent[b];
            int o = (int)((pos[3 * b] & 1) | ((pos[3 * b + 1] & 1) << 1) | ((pos[3 * b + 2] & 1) << 2));
            if (child[8 * p + o] != b) return fmt("block %lld: its parent %lld does not list it as a child", b, p);
        }
        if (is_leaf[b]) {
            for (int o = 0; o < 8; o++)
                if (child[8 * b + o] != -1) return fmt("leaf block %lld has a child", b);
        } else {
            for (int o = 0; o < 8; o++) {
                int c = child[8 * b + o];
                if (c < 0 || c >= n) return fmt("refined block %lld lacks child %lld", b, o);
                if (level[c] != level[b] + 1) return fmt("block %lld: child %lld is not one level finer", b, c);
                if (parent[c] != b) return fmt("block %lld: child %lld names another parent", b, c);
                if (pos[3 * c] != 2 * pos[3 * b] + (o & 1) || pos[3 * c + 1] != 2 * pos[3 * b + 1] + ((o >> 1) & 1) ||
                    pos[3 * c + 2] != 2 * pos[3 * b + 2] + ((o >> 2) & 1))
                    return fmt("block %lld: child %lld is not in octant %lld", b, c, o);
            }
        }
    }
    std::vector<int> base_at((size_t)nbase * nbase * nbase, -1);
    for (int b = 0; b < n; b++)
        if (level[b] == 0) base_at[(pos[3 * b + 2] * nbase + pos[3 * b + 1]) * nbase + pos[3 * b]] = b;

    // leaves in depth-first (Morton) order; canonical = order in the block list
    std::vector<int> canon_of_block(n, -1);
    int nleaf = 0;
    for (int b = 0; b < n; b++)
        if (is_leaf[b]) canon_of_block[b] = nleaf++;
    std::vector<int> internal_of_block(n, -1);
    t.leaves.clear();
    t.leaves.reserve(nleaf);
    std::function<void(int)> dfs_block = [&](int b) {
        if (is_leaf[b]) {
            internal_of_block[b] = (int)t.leaves.size();
            LeafInfo li{};
            for (int d = 0; d < 3; d++) li.lo[d] = lo[3 * b + d];
            li.h = box / ((double)((int64_t)nbase << level[b]) * kNB);
            li.canon = canon_of_block[b];
            t.leaves.push_back(li);
            return;
        }
        for (int o = 0; o < 8; o++) dfs_block(child[8 * b + o]);
    };
    std::function<void(int, int64_t, int64_t, int64_t)> dfs_virtual = [&](int depth, int64_t ix, int64_t iy,
                                                                          int64_t iz) {
        if (depth == vlev) {
            dfs_block(base_at[(iz * nbase + iy) * nbase + ix]);
            return;
        }
        for (int o = 0; o < 8; o++)
            dfs_virtual(depth + 1, 2 * ix + (o & 1), 2 * iy + ((o >> 1) & 1), 2 * iz + ((o >> 2) & 1));
    };
    dfs_virtual(0, 0, 0, 0);
    if ((int)t.leaves.size() != nleaf) return "some blocks are not reachable from the base lattice";
    t.internal_of_canon.assign(nleaf, -1);
    for (int f = 0; f < nleaf; f++) t.internal_of_canon[t.leaves[f].canon] = f;

    // breadth-first node list
    std::vector<Desc> nodes;
    nodes.reserve((size_t)nleaf * 73 + (size_t)n + 16);
    auto block_desc = [&](int b, int depth) {
        return Desc{(uint8_t)(is_leaf[b] ? LEAF_BLOCK : PARENT_BLOCK), depth, pos[3 * b], pos[3 * b + 1],
                    pos[3 * b + 2], b, 0};
    };
    if (vlev == 0)
        nodes.push_back(block_desc(base_at[0], 0));
    else
        nodes.push_back(Desc{VIRTUAL, 0, 0, 0, 0, -1, 0});
    t.child.clear();
    t.flags.clear();
    t.parent.assign(1, -1);
    int maxd = 0;
    for (size_t i = 0; i < nodes.size(); i++) {
        Desc d = nodes[i];
        int32_t first = (int32_t)nodes.size();
        int32_t flag = 0;
        switch (d.kind) {
            case VIRTUAL:
                for (int o = 0; o < 8; o++) {
                    int64_t cx = 2 * d.ix + (o & 1), cy = 2 * d.iy + ((o >> 1) & 1), cz = 2 * d.iz + ((o >> 2) & 1);
                    if (d.depth + 1 == vlev)
                        nodes.push_back(block_desc(base_at[(cz * nbase + cy) * nbase + cx], d.depth + 1));
                    else
                        nodes.push_back(Desc{VIRTUAL, d.depth + 1, cx, cy, cz, -1, 0});
                }
                break;
            case PARENT_BLOCK:
                for (int o = 0; o < 8; o++) nodes.push_back(block_desc(child[8 * d.ref + o], d.depth + 1));
                break;
            case LEAF_BLOCK: {
                int f = internal_of_block[d.ref];
                t.leaves[f].block_node = (int)i;
                t.leaves[f].oct_first = first;
                for (int o = 0; o < 8; o++)
                    nodes.push_back(Desc{OCTANT, d.depth + 1, 2 * d.ix + (o & 1), 2 * d.iy + ((o >> 1) & 1),
                                         2 * d.iz + ((o >> 2) & 1), f, o});
                break;
            }
            case OCTANT:
                if (d.sub == 0) t.leaves[d.ref].bot_first = first;
                for (int o = 0; o < 8; o++)
                    nodes.push_back(Desc{BOTTOM, d.depth + 1, 2 * d.ix + (o & 1), 2 * d.iy + ((o >> 1) & 1),
                                         2 * d.iz + ((o >> 2) & 1), d.ref, d.sub * 8 + o});
                break;
            case BOTTOM:
                first = (int32_t)((int64_t)d.ref * kCellsPerBlock + 8 * d.sub);
                flag = FLAG_BOTTOM;
                if (d.depth > maxd) maxd = d.depth;
                break;
        }
        if (nodes.size() > (size_t)INT32_MAX / 2) return "grid too large for 32-bit node ids";
        while (t.parent.size() < nodes.size()) t.parent.push_back((int32_t)i);
        t.child.push_back(first);
        t.flags.push_back(flag);
    }
    t.n_nodes = (int64_t)nodes.size();
    t.max_depth = maxd;
    t.root = 0;
    t.key.resize(nodes.size());
    t.geom.resize(nodes.size() * 4);
    for (size_t i = 0; i < nodes.size(); i++) {
        const Desc &d = nodes[i];
        t.key[i] = make_key(d.depth, d.ix, d.iy, d.iz);
        double l = box / (double)((int64_t)1 << d.depth);
        t.geom[4 * i + 0] = box_lo[0] + ((double)d.ix + 0.5) * l;
        t.geom[4 * i + 1] = box_lo[1] + ((double)d.iy + 0.5) * l;
        t.geom[4 * i + 2] = box_lo[2] + ((double)d.iz + 0.5) * l;
        t.geom[4 * i + 3] = l;
    }
    // nodes above the leaf blocks (virtual, parent blocks): their moments come
    // from the leaf blocks below them
    t.combine_nodes.clear();
    for (size_t i = 0; i < nodes.size(); i++)
        if (nodes[i].kind == VIRTUAL || nodes[i].kind == PARENT_BLOCK) t.combine_nodes.push_back((int32_t)i);
    // leaves are numbered depth-first, so the leaf blocks below any node form
    // one contiguous range of leaf ordinals
    std::vector<int32_t> lo_leaf(nodes.size(), INT32_MAX), hi_leaf(nodes.size(), -1), n_below(nodes.size(), 0);
    for (int f = 0; f < nleaf; f++)
        for (int32_t a = t.parent[t.leaves[f].block_node]; a >= 0; a = t.parent[a]) {
            lo_leaf[a] = std::min(lo_leaf[a], (int32_t)f);
            hi_leaf[a] = std::max(hi_leaf[a], (int32_t)f);
            n_below[a]++;
        }
    t.combine_range.assign(t.combine_nodes.size() * 2, 0);
    for (size_t q = 0; q < t.combine_nodes.size(); q++) {
        const int32_t a = t.combine_nodes[q];
        if (hi_leaf[a] < 0 || hi_leaf[a] - lo_leaf[a] + 1 != n_below[a]) return "leaf order is not depth-first";
        t.combine_range[2 * q + 0] = lo_leaf[a];
        t.combine_range[2 * q + 1] = hi_leaf[a] + 1;
    }
    return "";
}

}  // namespace bh
