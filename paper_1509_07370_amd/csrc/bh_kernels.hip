// HIP kernels for gfx950 (CDNA4, wave64) of the Barnes-Hut potential path.
//
//   moments_leaf_kernel    one workgroup per leaf block: cells -> 64 bottom nodes
//                          -> 8 octants -> block node by lane shuffles (fp64)
//   moments_upper_kernel   the nodes above the leaf blocks, one workgroup per
//                          node, each from the leaf blocks below it; beside
//                          them, the placement of the walks' dispatch order
//   walk_kernel            one wavefront per 64-cell group: breadth-limited
//                          depth-first traversal with an LDS stack of sibling
//                          sets; 64 lanes test 8 sibling sets at once, the
//                          group vote is exact and O(1) per node (see below)
//   scan kernels           CSR offsets of the interaction lists
//   potential kernels      one wavefront per group, one lane per cell; far
//                          nodes and near cells staged through LDS in tiles of
//                          64 and read back as wave-wide broadcasts
//   direct_kernel          exact fp64 O(N^2) reference
#include <hip/hip_runtime.h>

#include "bh_device.h"
#include "bh_ewald.h"
#include "bh_internal.h"

namespace bh {

// ---------------------------------------------------------------- helpers

struct MomOut {
    double *mom;
    WalkRec32 *w32;
    WalkRec64 *w64;
    FarRec32 *f32;
    double *s;     // [n] sum m |r - X|^2
    double *brow;  // [n_leaf][kBlockRow] leaf-ordered copies of the block nodes' rows
};

// Write every derived record of node `id` from its fp64 moments (and, for a
// leaf block node, the copy of its row at leaf ordinal `leaf`).
__device__ void store_node(const MomOut &o, int id, double M, double X, double Y, double Z, const double *Q, double S,
                           const double *geom, int child, int sflags, double mmax = 0.0, int leaf = -1) {
#pragma clang fp contract(off)
    double cx = geom[0], cy = geom[1], cz = geom[2], l = geom[3];
    double q[6];
    double delta;
    int flags = sflags;
    if (M > 0.0) {
        double ex = X - cx, ey = Y - cy, ez = Z - cz;
        delta = sqrt(ex * ex + ey * ey + ez * ez);
        for (int c = 0; c < 6; c++) q[c] = Q[c];
    } else {
        X = cx;
        Y = cy;
        Z = cz;
        delta = 0.0;
        for (int c = 0; c < 6; c++) q[c] = 0.0;
        flags |= FLAG_EMPTY;
        M = 0.0;
        S = 0.0;
    }
    o.s[id] = S;
    double *mo = o.mom + (int64_t)id * kMom;
    mo[0] = X;
    mo[1] = Y;
    mo[2] = Z;
    mo[3] = M;
    for (int c = 0; c < 6; c++) mo[4 + c] = q[c];
    mo[10] = delta;
    mo[11] = mmax;
    if (leaf >= 0) {
        double *b = o.brow + (int64_t)leaf * kBlockRow;
        b[0] = X;
        b[1] = Y;
        b[2] = Z;
        b[3] = M;
        for (int c = 0; c < 6; c++) b[4 + c] = q[c];
        b[10] = S;
        b[11] = 0.0;
    }
    WalkRec32 w;
    w.x = (float)X;
    w.y = (float)Y;
    w.z = (float)Z;
    w.delta = (float)delta;
    w.l = (float)l;
    w.child = child;
    w.flags = flags;
    w.pad = 0;
    o.w32[id] = w;
    WalkRec64 w2;
    w2.x = X;
    w2.y = Y;
    w2.z = Z;
    w2.delta = delta;
    w2.l = l;
    w2.child = child;
    w2.flags = flags;
    o.w64[id] = w2;
    FarRec32 f;
    f.x = (float)X;
    f.y = (float)Y;
    f.z = (float)Z;
    f.m = (float)M;
    f.a = (float)(0.5 * q[0]);
    f.b = (float)(0.5 * q[1]);
    f.f = (float)(0.5 * q[2]);
    f.c = (float)q[3];
    f.d = (float)q[4];
    f.e = (float)q[5];
    f.s = (float)S;
    f.pad1 = 0.f;
    o.f32[id] = f;
}

// ---------------------------------------------------------------- moments

// Butterfly sum / max over the 8 lanes of an aligned group of 8 (every lane
// ends with the same bits: each level adds the same two partial sums), with
// the lane exchanges as DPP moves rather than LDS permutes: lane ^ 1 and
// lane ^ 2 are quad permutations; after them every lane of a quad holds the
// quad's result, so the last level may take the other quad's from lane 7 - i
// (the half-row mirror) instead of lane ^ 4 -- the same value.
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
    const uint64_t u = (uint64_t)__double_as_longlong(v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)u, CTRL, 0xF, 0xF, false);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)(u >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}
constexpr int kDppXor1 = 0xB1;        // quad_perm [1, 0, 3, 2]
constexpr int kDppXor2 = 0x4E;        // quad_perm [2, 3, 0, 1]
constexpr int kDppHalfMirror = 0x141;  // row_half_mirror: lane 7 - i within each 8
__device__ __forceinline__ double sum8(double v) {
    v += dpp_f64<kDppXor1>(v);
    v += dpp_f64<kDppXor2>(v);
    v += dpp_f64<kDppHalfMirror>(v);
    return v;
}
__device__ __forceinline__ double max8(double v) {
    double u = dpp_f64<kDppXor1>(v);
    v = u > v ? u : v;
    u = dpp_f64<kDppXor2>(v);
    v = u > v ? u : v;
    u = dpp_f64<kDppHalfMirror>(v);
    return u > v ? u : v;
}

// One node from its 8 children held by the 8 lanes of a group (child c in
// lane c): M, centre of mass, quadrupole and S = sum m |r - X|^2 about it by
// the parallel-axis rule.  Cells enter as children with Q = 0 and S = 0.
// Every lane of the group gets the node.
__device__ __forceinline__ void combine_lanes(double m, double x, double y, double z, const double *qc, double sc,
                                              double &M, double &X, double &Y, double &Z, double *Q, double &S) {
#pragma clang fp contract(off)
    M = sum8(m);
    const double sx = sum8(m * x), sy = sum8(m * y), sz = sum8(m * z);
    X = M > 0.0 ? sx / M : 0.0;
    Y = M > 0.0 ? sy / M : 0.0;
    Z = M > 0.0 ? sz / M : 0.0;
    const double dx = x - X, dy = y - Y, dz = z - Z;
    const double r2 = dx * dx + dy * dy + dz * dz;
    Q[0] = sum8(qc[0] + m * (3.0 * dx * dx - r2));
    Q[1] = sum8(qc[1] + m * (3.0 * dy * dy - r2));
    Q[2] = sum8(qc[2] + m * (3.0 * dz * dz - r2));
    Q[3] = sum8(qc[3] + m * (3.0 * dx * dy));
    Q[4] = sum8(qc[4] + m * (3.0 * dx * dz));
    Q[5] = sum8(qc[5] + m * (3.0 * dy * dz));
    S = sum8(sc + m * r2);
}

// ---------------------------------------------------------------- dispatch schedule
//
// The fused walks dispatch their groups heaviest first (the longest start
// first and short ones fill the end of the launch), in the order of the work
// that the previous fused walk recorded per group.  The upward pass builds
// that order as a counting sort over 256 bins of log2 cost (1/8 octave
// each), with no launch of its own: the leaf-block kernel counts each block's
// groups into a histogram, and the upper-node kernel, once the histogram is
// complete, places every group at its bin's start plus a cursor taken with an
// atomic.  The last workgroup of the placement to finish returns the
// histogram and the cursors to zero, so that every pass -- also each replay
// of a captured graph -- starts from zero.  The order within a bin follows
// the atomics; it decides which wavefront computes a group, not what it
// computes.
struct SchedArgs {
    const uint32_t *cost;  // [n_units] from the last fused walk; NULL: no schedule in this pass
    int *hist;             // [256] bin counts (zero between passes)
    int *cursor;           // [256] placement cursors (zero between passes)
    int *done;             // workgroups of the placement that have finished (zero between passes)
    int32_t *order;        // [n_units] dispatch order of the 64-cell octants
    int64_t n_units;
    int parts;             // workgroups of the placement, the first ones of the upper-node launch
};

__device__ __forceinline__ int cost_bin(uint32_t c) {
    const int b = (int)(log2f((float)c + 1.0f) * 8.0f);
    return 255 - (b > 255 ? 255 : b);
}

__device__ __forceinline__ int wave_inclusive_scan(int v) {
    const int lane = (int)(threadIdx.x & 63);
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int u = __shfl_up(v, d);
        if (lane >= d) v += u;
    }
    return v;
}

// Lanes of a wavefront grouped by equal key: each active lane gets the lowest
// lane with its key (the leader), its rank among those lanes and their
// number.  One pass per distinct key; called by the whole wavefront.
__device__ __forceinline__ void wave_key_groups(int key, bool active, int &leader, int &rank, int &count) {
    const int lane = (int)(threadIdx.x & 63);
    const uint64_t below = (1ull << lane) - 1ull;
    uint64_t todo = __ballot(active);
    leader = lane;
    rank = 0;
    count = 0;
    while (todo) {
        const int l = __ffsll((unsigned long long)todo) - 1;
        const int k = __shfl(key, l);
        const bool mine = active && key == k;
        const uint64_t same = __ballot(mine);
        if (mine) {
            leader = l;
            rank = __popcll(same & below);
            count = __popcll(same);
        }
        todo &= ~same;
    }
}

// Histogram of the 8 groups of leaf block f (first 8 lanes of a wavefront;
// one atomic per distinct bin).  Called by whole wavefronts.
__device__ __forceinline__ void sched_count(const SchedArgs &sa, int f, int lane) {
    const bool act = lane < 8;
    const int b = cost_bin(sa.cost[(int64_t)f * 8 + (act ? lane : 0)]);
    int leader, rank, count;
    wave_key_groups(b, act, leader, rank, count);
    if (act && leader == lane) atomicAdd(&sa.hist[b], count);
}

// Places the groups [q0, q1) (one 256-thread workgroup): exclusive scan of
// the complete histogram into bin starts, then per wavefront one atomic per
// distinct bin reserves consecutive slots.  The workgroup that finishes last
// clears the histogram, the cursors and the counter: every other workgroup's
// reads of the histogram and cursor atomics have returned before its count
// is taken, so nothing is read after the clearing.
__device__ void sched_place(const SchedArgs &sa, int64_t q0, int64_t q1, int *start, int *wave_total) {
    const int t = threadIdx.x, lane = t & 63;
    const int v = sa.hist[t];
    const int incl = wave_inclusive_scan(v);
    if (lane == 63) wave_total[t >> 6] = incl;
    __syncthreads();
    int base = incl - v;
    for (int w = 0; w < (t >> 6); w++) base += wave_total[w];
    start[t] = base;
    __syncthreads();
    for (int64_t qb = q0; qb < q1; qb += 256) {
        const int64_t q = qb + t;
        const bool act = q < q1;
        const int b = cost_bin(sa.cost[act ? q : q0]);
        int leader, rank, count;
        wave_key_groups(b, act, leader, rank, count);
        int old = 0;
        if (act && leader == lane) old = atomicAdd(&sa.cursor[b], count);
        old = __shfl(old, leader);
        if (act) sa.order[start[b] + old + rank] = (int32_t)q;
    }
    __shared__ int last;
    __syncthreads();
    if (t == 0) last = atomicAdd(sa.done, 1) == sa.parts - 1;
    __syncthreads();
    if (last) {
        sa.hist[t] = 0;
        sa.cursor[t] = 0;
        if (t == 0) *sa.done = 0;
    }
}

// In-block part of the upward pass, one 512-thread workgroup per leaf block.
// Thread t owns cell t of the block in Morton order, so the 8 cells of bottom
// node b sit in lanes 8b..8b+7 and combine by lane shuffles; the 64 bottom
// nodes then combine into the 8 octants and the block node in the first
// wavefront.
__global__ __launch_bounds__(512) void moments_leaf_kernel(const double *__restrict__ rho,
                                                           const LeafInfo *__restrict__ leaves,
                                                           const double *__restrict__ geom,
                                                           const int32_t *__restrict__ child_arr, MomOut out,
                                                           double4 *__restrict__ cell64, float4 *__restrict__ cell32,
                                                           int *__restrict__ flags, int epoch, SchedArgs sa) {
#pragma clang fp contract(off)
    __shared__ double bM[64], bX[64], bY[64], bZ[64], bQ[64][6], bS[64], bmax[64];
    const int f = blockIdx.x;
    const int t = threadIdx.x;
    const LeafInfo L = leaves[f];
    int i, j, k;
    demorton9(t, i, j, k);
    const double r = rho[(int64_t)L.canon * kCellsPerBlock + k * 64 + j * 8 + i];
    if (!(r >= 0.0) || !isfinite(r)) atomicMax(flags, epoch);
    const double h = L.h;
    const double mass = r * (h * h * h);
    const double x = L.lo[0] + (i + 0.5) * h;
    const double y = L.lo[1] + (j + 0.5) * h;
    const double z = L.lo[2] + (k + 0.5) * h;
    const int64_t c = (int64_t)f * kCellsPerBlock + t;
    cell64[c] = make_double4(x, y, z, mass);
    cell32[c] = make_float4((float)x, (float)y, (float)z, (float)mass);
    {  // bottom node t >> 3 from its 8 cells
        const double q0[6] = {0, 0, 0, 0, 0, 0};
        double M, X, Y, Z, Q[6], S;
        combine_lanes(mass, x, y, z, q0, 0.0, M, X, Y, Z, Q, S);
        const double mx = max8(mass);
        if ((t & 7) == 0) {
            const int b = t >> 3, id = L.bot_first + b;
            store_node(out, id, M, X, Y, Z, Q, S, geom + 4 * (int64_t)id, child_arr[id], FLAG_BOTTOM, mx);
            bM[b] = M;
            bX[b] = M > 0.0 ? X : geom[4 * (int64_t)id + 0];
            bY[b] = M > 0.0 ? Y : geom[4 * (int64_t)id + 1];
            bZ[b] = M > 0.0 ? Z : geom[4 * (int64_t)id + 2];
            for (int q = 0; q < 6; q++) bQ[b][q] = M > 0.0 ? Q[q] : 0.0;
            bS[b] = M > 0.0 ? S : 0.0;
            bmax[b] = mx;
        }
    }
    __syncthreads();
    if (t >= 64) {
        if (sa.cost && t < 128) sched_count(sa, f, t - 64);  // the dispatch schedule's histogram
        return;
    }
    // octant t >> 3 from its 8 bottom nodes (lane t holds bottom node t)
    double M, X, Y, Z, Q[6], S;
    combine_lanes(bM[t], bX[t], bY[t], bZ[t], bQ[t], bS[t], M, X, Y, Z, Q, S);
    const double mx = max8(bmax[t]);
    const int o = t >> 3;
    const int oid = L.oct_first + o;
    if ((t & 7) == 0) store_node(out, oid, M, X, Y, Z, Q, S, geom + 4 * (int64_t)oid, child_arr[oid], 0, mx);
    // block node from the 8 octants: lane c of the first group takes octant c
    const double e = M > 0.0 ? 1.0 : 0.0;
    const double oX = M > 0.0 ? X : geom[4 * (int64_t)oid + 0];
    const double oY = M > 0.0 ? Y : geom[4 * (int64_t)oid + 1];
    const double oZ = M > 0.0 ? Z : geom[4 * (int64_t)oid + 2];
    const int src = 8 * (t & 7);
    double oq[6];
    for (int q = 0; q < 6; q++) oq[q] = __shfl(Q[q] * e, src, 64);
    double BM, BX, BY, BZ, BQ[6], BS;
    combine_lanes(__shfl(M, src, 64), __shfl(oX, src, 64), __shfl(oY, src, 64), __shfl(oZ, src, 64), oq,
                  __shfl(S * e, src, 64), BM, BX, BY, BZ, BQ, BS);
    if (t != 0) return;
    const int node = L.block_node;
    store_node(out, node, BM, BX, BY, BZ, BQ, BS, geom + 4 * (int64_t)node, child_arr[node], 0, 0.0, f);
}

// N block-wide sums of one double per thread (256 threads) at once, each in
// a fixed order: wavefront butterflies, then the four wavefront totals in
// order; one pair of barriers for all of them.  Every thread gets the same
// values.  red: N x 4 doubles of LDS.
template <int N>
__device__ __forceinline__ void block_sums256(double (&v)[N], double (*red)[4]) {
#pragma unroll
    for (int k = 0; k < N; k++) {
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) v[k] += __shfl_xor(v[k], o, 64);
    }
    __syncthreads();
    if ((threadIdx.x & 63) == 0) {
#pragma unroll
        for (int k = 0; k < N; k++) red[k][threadIdx.x >> 6] = v[k];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < N; k++) v[k] = ((red[k][0] + red[k][1]) + red[k][2]) + red[k][3];
}

// Nodes above the leaf blocks (virtual and parent-block nodes), one
// 256-thread workgroup per node, all at once: a node's moments are those of
// the leaf blocks below it -- a contiguous range of leaf ordinals -- combined
// directly (mass and centre of mass, then the quadrupole about it by the
// parallel-axis rule), so no node waits for its children.  The leaf blocks'
// rows are the leaf-ordered copies moments_leaf_kernel writes (one load per
// row, no lookup of the block's node id).
__global__ __launch_bounds__(256) void moments_upper_kernel(const int32_t *__restrict__ nodes,
                                                            const int32_t *__restrict__ range,
                                                            const double *__restrict__ geom,
                                                            const int32_t *__restrict__ child_arr, MomOut out,
                                                            SchedArgs sa) {
#pragma clang fp contract(off)
    __shared__ double red[7][4];
    if (sa.cost && (int)blockIdx.x < sa.parts) {  // a share of the dispatch schedule's placement
        __shared__ int start[256], wave_total[4];
        const int64_t n = sa.n_units, p = blockIdx.x;
        sched_place(sa, n * p / sa.parts, n * (p + 1) / sa.parts, start, wave_total);
        return;
    }
    const int q = blockIdx.x - (sa.cost ? sa.parts : 0);
    const int id = nodes[q];
    const int f0 = range[2 * q], f1 = range[2 * q + 1];
    double p1[4] = {0.0, 0.0, 0.0, 0.0};  // m, m x, m y, m z
#pragma unroll 4
    for (int f = f0 + (int)threadIdx.x; f < f1; f += 256) {
        const double *r = out.brow + (int64_t)f * kBlockRow;
        const double mb = r[3];
        p1[0] += mb;
        p1[1] += mb * r[0];
        p1[2] += mb * r[1];
        p1[3] += mb * r[2];
    }
    block_sums256(p1, red);
    const double M = p1[0];
    const double X = M > 0.0 ? p1[1] / M : 0.0, Y = M > 0.0 ? p1[2] / M : 0.0, Z = M > 0.0 ? p1[3] / M : 0.0;
    double qa[6] = {0, 0, 0, 0, 0, 0}, sa_ = 0.0;
#pragma unroll 4
    for (int f = f0 + (int)threadIdx.x; f < f1; f += 256) {
        const double *r = out.brow + (int64_t)f * kBlockRow;
        const double mb = r[3];
        const double dx = r[0] - X, dy = r[1] - Y, dz = r[2] - Z;
        const double r2 = dx * dx + dy * dy + dz * dz;
        sa_ += r[10] + mb * r2;
        qa[0] += r[4] + mb * (3.0 * dx * dx - r2);
        qa[1] += r[5] + mb * (3.0 * dy * dy - r2);
        qa[2] += r[6] + mb * (3.0 * dz * dz - r2);
        qa[3] += r[7] + mb * (3.0 * dx * dy);
        qa[4] += r[8] + mb * (3.0 * dx * dz);
        qa[5] += r[9] + mb * (3.0 * dy * dz);
    }
    double p2[7] = {qa[0], qa[1], qa[2], qa[3], qa[4], qa[5], sa_};
    block_sums256(p2, red);
    if (threadIdx.x == 0) store_node(out, id, M, X, Y, Z, p2, p2[6], geom + 4 * (int64_t)id, child_arr[id], 0);
}

hipError_t launch_moments(const bh_grid *g, bh_moments *m, const double *rho, hipStream_t s, int fixed_epoch,
                          bool schedule) {
    MomOut o{m->d_mom, m->d_w32, m->d_w64, m->d_f32, m->d_s, m->d_brow};
    const int nleaf = (int)g->topo.leaves.size();
    const int epoch = fixed_epoch > 0 ? fixed_epoch : ++m->mom_epoch;
    SchedArgs sa{};
    if (schedule) {
        if (g->n_units != 8 * (int64_t)nleaf) return hipErrorInvalidValue;
        // one placement workgroup per 256 octants, launched beside the node workgroups
        sa = SchedArgs{m->d_cost, m->d_sched, m->d_sched + 256, m->d_sched + 512, m->d_order, g->n_units,
                       (int)((g->n_units + 255) / 256)};
    }
    hipLaunchKernelGGL(moments_leaf_kernel, dim3(nleaf), dim3(512), 0, s, rho, g->d_leaves, g->d_geom, g->d_child, o,
                       m->d_cell64, m->d_cell32, m->d_flags, epoch, sa);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t blocks = (int64_t)g->topo.combine_nodes.size() + sa.parts;
    if (blocks == 0) return hipSuccess;
    hipLaunchKernelGGL(moments_upper_kernel, dim3((unsigned)blocks), dim3(256), 0, s, g->d_combine,
                       g->d_combine_range, g->d_geom, g->d_child, o, sa);
    return hipGetLastError();
}

// ---------------------------------------------------------------- walk

template <typename real>
struct Prec;
template <>
struct Prec<float> {
    using Rec = WalkRec32;
    using V4 = float4;
};
template <>
struct Prec<double> {
    using Rec = WalkRec64;
    using V4 = double4;
};

// min over k in [0, n) of |fl(x0 + k h - X)|.  x0 + k h is exact (dyadic), and
// fl(a - X) is monotone in a, so the minimum sits at one of the two lattice
// points around X; both are evaluated exactly as a per-cell test would.  The
// bracketing index needs only to be right to within one: (X - x0) * (1/h)
// instead of a division can move floor() by one only where X is within
// rounding of a lattice point, and that point is still one of the two
// candidates.
template <typename real>
__device__ __forceinline__ real nearest_gap(real x0, real h, real hinv, real X, int n) {
#pragma clang fp contract(off)
    real t = (X - x0) * hinv;
    int k = (int)floor(t);
    k = k < 0 ? 0 : (k > n - 1 ? n - 1 : k);
    int k2 = k + 1 > n - 1 ? n - 1 : k + 1;
    real d1 = (x0 + (real)k * h) - X;
    real d2 = (x0 + (real)k2 * h) - X;
    d1 = d1 < 0 ? -d1 : d1;
    d2 = d2 < 0 ? -d2 : d2;
    return d1 < d2 ? d1 : d2;
}


// distance from X to the interval [lo, hi] along one axis
template <typename real>
__device__ __forceinline__ real cube_gap(real lo, real hi, real X) {
#pragma clang fp contract(off)
    const real below = lo - X, above = X - hi;
    return below > (real)0 ? below : (above > (real)0 ? above : (real)0);
}

// The cell-centre lattice of one group: the first centre per axis and the
// number of centres per axis.  Groups are aligned Morton runs of gcells
// cells inside a block (Morton bit 0 = x): 32 -> 4x4x2, 64 -> 4x4x4,
// 128 -> 8x4x4, 256 -> 8x8x4, 512 -> 8x8x8 cells.
template <typename real>
struct GroupBox {
    real x0[3];
    int n[3];
};

template <typename real>
__device__ __forceinline__ GroupBox<real> group_box(const LeafInfo &L, int gcells, int run) {
    int i0, j0, k0;
    demorton9(run * gcells, i0, j0, k0);
    GroupBox<real> b;
    b.n[0] = gcells >= 128 ? 8 : 4;
    b.n[1] = gcells >= 256 ? 8 : 4;
    b.n[2] = gcells >= 512 ? 8 : (gcells >= 64 ? 4 : 2);
    b.x0[0] = (real)(L.lo[0] + (i0 + 0.5) * L.h);
    b.x0[1] = (real)(L.lo[1] + (j0 + 0.5) * L.h);
    b.x0[2] = (real)(L.lo[2] + (k0 + 0.5) * L.h);
    return b;
}

// Groups per leaf block and the group (within the block) of octant `sub`.
__device__ __forceinline__ int groups_per_leaf(int gcells) { return kCellsPerBlock / gcells; }

__device__ __forceinline__ float clamp_theta(float th) {
    if (!(th == th)) th = 1e-3f;
    return th < 1e-3f ? 1e-3f : (th > 1.0f ? 1.0f : th);
}
__device__ __forceinline__ float group_theta(const WalkArgs &a, int64_t canon_group) {
    return clamp_theta(a.theta_group[canon_group]);
}

// Group walk state of one wavefront.  The group vote of the potential kernel
// (all cells of the group accept) needs, per node, the minimum over the
// group's cells of d^2.  The group is an axis-aligned lattice of cell
// centres, so that minimum separates per axis: the cell whose per-axis gaps
// are each minimal has the smallest rounded d^2 too (rounding is monotone).
// One lane therefore decides one node exactly as per-cell tests would, and a
// step tests the 64 children of up to 8 opened nodes.  The LDS stack holds
// the first-child ids of opened nodes; it pops 8 entries while it is short
// and 1 entry (plain depth-first order, growth <= 7 per level) once it passes
// k8_threshold, so it never exceeds k8_threshold + 56 + 7 (max_depth + 1) + 1
// < kWalkStackCap.
// GM = 1: one group (any size); its cells may span several wavefronts, each
// of which walks the same tree with the same decisions.
// GM = 2: two 32-cell groups on one wavefront (the halves z < 2 and z >= 2 of
// a 4x4x4 octant; lanes 0-31 and 32-63).  Each stack entry carries a 2-bit
// mask of the groups that still need its sibling set (entry = child * 4 +
// mask); a node is tested for each group in its mask, and its outcome per
// group goes to `acc` / `nr` as masks (bit 0: lanes 0-31's group).
// MAC 0: the exact vote of every cell of the group (O(1) per node, above);
// MAC 1: the paper's test between a node and a region -- the smallest
// distance from the node's centre of mass to the group's cube (cell faces);
// MAC 2: the periodic box's nearest-image distances.
template <typename real, int MAC = 0, int GM = 1>
struct Walker {
    using Rec = typename Prec<real>::Rec;
    const Rec *nodes;
    int *stk;
    int size;
    int k8;
    real h, hinv;
    GroupBox<real> box;
    real z0b;          // GM 2: first z centre of the second group
    real inv, invb;    // 1/theta of the group(s)
    real box_l, box_inv;  // MAC 2 only
    bool overflow;

    // MAC 2: min over the group's n centres x0 + k h on one axis of the
    // nearest-image distance to X
    __device__ real periodic_gap(real x0_, int n, real X) const {
#pragma clang fp contract(off)
        const real c = x0_ + (real)0.5 * (real)(n - 1) * h;
        const real Xn = X - box_l * rint((X - c) * box_inv);  // image nearest the centre
        const real Xo = Xn < c ? Xn + box_l : Xn - box_l;       // the next one on the other side
        const real g1 = nearest_gap<real>(x0_, h, hinv, Xn, n), g2 = nearest_gap<real>(x0_, h, hinv, Xo, n);
        return g1 < g2 ? g1 : g2;
    }
    __device__ real axis_gap(real x0_, int n, real X) const {
#pragma clang fp contract(off)
        if constexpr (MAC == 1) {  // cube [first centre - h/2, last centre + h/2]
            const real half = (real)0.5 * h;
            return cube_gap<real>(x0_ - half, (x0_ + (real)(n - 1) * h) + half, X);
        } else if constexpr (MAC == 2) {
            return periodic_gap(x0_, n, X);
        } else {
            return nearest_gap<real>(x0_, h, hinv, X, n);
        }
    }

    // g0: canonical index of the (first) group, for the per-group theta
    __device__ void init(const WalkArgs &a, const LeafInfo &L, const GroupBox<real> &b, int64_t g0, int *stack,
                         int lane) {
        nodes = (const Rec *)a.nodes;
        stk = stack;
        k8 = a.k8_threshold;
        overflow = false;
        h = (real)L.h;
        hinv = (real)1 / h;
        box = b;
        if constexpr (GM == 2) z0b = b.x0[2] + (real)2 * h;
        if constexpr (MAC == 2) {
            box_l = (real)a.box;
            box_inv = (real)(1.0 / a.box);
        }
        if (a.theta_group) {
            inv = (real)1 / (real)group_theta(a, g0);
            if constexpr (GM == 2) invb = (real)1 / (real)group_theta(a, g0 + 1);
        } else {
            if (sizeof(real) == 4)
                inv = (real)(1.0f / (float)a.theta);
            else
                inv = (real)(1.0 / a.theta);
            invb = inv;
        }
        size = 0;
        const Rec root = nodes[a.root];
        if (!(root.flags & FLAG_EMPTY)) {
            if (lane == 0) stk[0] = GM == 2 ? root.child * 4 + 3 : root.child;
            size = 1;
        }
        wave_lds_sync();
    }

    // One step.  Per lane: id of the tested node, and whether it was accepted
    // (far) or is a rejected bottom node (near) -- for GM 2 as masks of the
    // two groups.  Opened nodes are pushed.
    __device__ void step(int lane, int &id, int &acc, int &nr, int &cid) {
        const int k = size <= k8 ? (size < 8 ? size : 8) : 1;
        const int slot = lane >> 3;
        const bool active = slot < k;
        int mask = 1;
        id = 0;
        if (active) {
            const int e = stk[size - 1 - slot];
            if constexpr (GM == 2) {
                id = (e >> 2) + (lane & 7);
                mask = e & 3;
            } else {
                id = e + (lane & 7);
            }
        }
        size -= k;
        wave_lds_sync();
        acc = 0;
        nr = 0;
        cid = 0;
        bool op = false;
        int ch = 0;
        if (active) {
            const Rec r = nodes[id];
            if (!(r.flags & FLAG_EMPTY)) {
#pragma clang fp contract(off)
                const real dx = axis_gap(box.x0[0], box.n[0], r.x);
                const real dy = axis_gap(box.x0[1], box.n[1], r.y);
                const real dz = axis_gap(box.x0[2], box.n[2], r.z);
                const real dxy = dx * dx + dy * dy;
                const real d2 = dxy + dz * dz;
                const real s = r.l * inv + r.delta;
                int fm = (mask & 1) && d2 > s * s ? 1 : 0;
                if constexpr (GM == 2) {
                    const real dzb = axis_gap(z0b, box.n[2], r.z);
                    const real d2b = dxy + dzb * dzb;
                    const real sb = r.l * invb + r.delta;
                    fm |= (mask & 2) && d2b > sb * sb ? 2 : 0;
                }
                acc = fm;
                const int om = mask & ~fm;
                if (om) {
                    if (r.flags & FLAG_BOTTOM) {
                        nr = om;
                        cid = r.child;  // a bottom node's first cell (internal order)
                    } else {
                        op = true;
                        ch = GM == 2 ? r.child * 4 + om : r.child;
                    }
                }
            }
        }
        const uint64_t mo = __ballot(op);
        if (op) {
            int p = size + lane_prefix(mo);
            if (p < kWalkStackCap)
                stk[p] = ch;
            else
                overflow = true;
        }
        size += __popcll(mo);
        if (size > kWalkStackCap) {
            overflow = true;
            size = 0;
        }
        wave_lds_sync();
    }

    __device__ void finish(const WalkArgs &a, int lane) {
        if (__ballot(overflow) != 0 && lane == 0) atomicMax(a.flags + 1, a.epoch);
    }
};

// One wavefront per group (internal group order: leaf in internal order, then
// the group's Morton run in the block), whatever the group size.
template <typename real, bool FILL>
__global__ __launch_bounds__(256) void walk_kernel(WalkArgs a) {
    __shared__ int stack[4][kWalkStackCap];
    const int w = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    const int64_t g = (int64_t)blockIdx.x * 4 + w;
    if (g >= a.n_groups) return;
    const int gpl = groups_per_leaf(a.gcells);
    const int f = (int)(g / gpl), run = (int)(g % gpl);
    const LeafInfo L = a.leaves[f];
    Walker<real> W;
    W.init(a, L, group_box<real>(L, a.gcells, run), (int64_t)L.canon * gpl + run, stack[w], lane);
    int64_t fbase = 0, nbase = 0;
    if (FILL) {
        fbase = a.far_off[g];
        nbase = a.near_off[g];
    }
    int nf = 0, nn = 0;
    while (W.size > 0) {
        int id, acc, nr, cid;
        W.step(lane, id, acc, nr, cid);
        const uint64_t mf = __ballot(acc);
        const uint64_t mn = __ballot(nr);
        if (FILL) {
            if (acc) a.far_out[fbase + nf + lane_prefix(mf)] = id;
            if (nr) a.near_out[nbase + nn + lane_prefix(mn)] = id;
        }
        nf += __popcll(mf);
        nn += __popcll(mn);
    }
    W.finish(a, lane);
    if (!FILL && lane == 0) {
        a.far_cnt[g] = nf;
        a.near_cnt[g] = nn;
    }
}

int walk_k8_threshold(int max_depth) { return kWalkStackCap - 64 - 7 * (max_depth + 1) - 8; }

static WalkArgs walk_args(const bh_grid *g, const bh_moments *m, double theta, const float *theta_group,
                          int precision, int epoch) {
    WalkArgs a{};
    a.nodes = precision == BH_FP64 ? (const void *)m->d_w64 : (const void *)m->d_w32;
    a.leaves = g->d_leaves;
    a.theta_group = theta_group;
    a.theta = theta;
    a.n_groups = g->n_groups;
    a.gcells = g->group_cells;
    a.n_units = g->n_units;
    a.root = g->topo.root;
    a.k8_threshold = walk_k8_threshold(g->topo.max_depth);
    a.epoch = epoch;
    a.flags = m->d_flags;
    a.child = g->d_child;
    return a;
}

hipError_t launch_walk(const bh_grid *g, const bh_moments *m, bh_lists *L, double theta, const float *theta_group,
                       int precision, bool fill, hipStream_t s) {
    WalkArgs a = walk_args(g, m, theta, theta_group, precision, m->walk_epoch);
    a.far_cnt = L->d_far_cnt;
    a.near_cnt = L->d_near_cnt;
    a.far_off = L->d_far_off;
    a.near_off = L->d_near_off;
    a.far_out = L->d_far;
    a.near_out = L->d_near;
    const int blocks = (int)((g->n_groups + 3) / 4);
    if (precision == BH_FP64) {
        if (fill)
            hipLaunchKernelGGL((walk_kernel<double, true>), dim3(blocks), dim3(256), 0, s, a);
        else
            hipLaunchKernelGGL((walk_kernel<double, false>), dim3(blocks), dim3(256), 0, s, a);
    } else {
        if (fill)
            hipLaunchKernelGGL((walk_kernel<float, true>), dim3(blocks), dim3(256), 0, s, a);
        else
            hipLaunchKernelGGL((walk_kernel<float, false>), dim3(blocks), dim3(256), 0, s, a);
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------- scan

constexpr int kScanBlock = 256;
constexpr int kScanItems = 4;
constexpr int kScanTile = kScanBlock * kScanItems;

__device__ __forceinline__ int64_t block_exclusive_scan(int64_t v, int64_t *sh, int64_t &total) {
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int off = 1; off < kScanBlock; off <<= 1) {
        int64_t add = t >= off ? sh[t - off] : 0;
        __syncthreads();
        sh[t] += add;
        __syncthreads();
    }
    total = sh[kScanBlock - 1];
    int64_t incl = sh[t];
    __syncthreads();
    return incl - v;
}

__global__ __launch_bounds__(kScanBlock) void scan_reduce_kernel(const int32_t *__restrict__ a,
                                                                 const int32_t *__restrict__ b, int64_t n,
                                                                 int64_t *__restrict__ partials, int nblocks) {
    __shared__ int64_t sh[kScanBlock];
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    int64_t sa = 0, sb = 0;
    for (int q = 0; q < kScanItems; q++) {
        if (base + q < n) {
            sa += a[base + q];
            sb += b[base + q];
        }
    }
    int64_t ta, tb;
    block_exclusive_scan(sa, sh, ta);
    block_exclusive_scan(sb, sh, tb);
    if (threadIdx.x == 0) {
        partials[blockIdx.x] = ta;
        partials[nblocks + blockIdx.x] = tb;
    }
}

// Scans the block sums, writes both list totals (end offsets) and gathers the
// walk and density flags into status[] for one host copy.
__global__ __launch_bounds__(kScanBlock) void scan_partials_kernel(int64_t *__restrict__ partials, int nblocks,
                                                                   int64_t *__restrict__ end_a,
                                                                   int64_t *__restrict__ end_b,
                                                                   const int *__restrict__ flags,
                                                                   int64_t *__restrict__ status) {
    __shared__ int64_t sh[kScanBlock];
    for (int which = 0; which < 2; which++) {
        int64_t *p = partials + (int64_t)which * nblocks;
        int64_t carry = 0;
        for (int base = 0; base < nblocks; base += kScanBlock) {
            int idx = base + threadIdx.x;
            int64_t v = idx < nblocks ? p[idx] : 0;
            int64_t tot;
            int64_t ex = block_exclusive_scan(v, sh, tot);
            if (idx < nblocks) p[idx] = ex + carry;
            carry += tot;
        }
        if (threadIdx.x == 0) {
            *(which == 0 ? end_a : end_b) = carry;
            status[which] = carry;
        }
    }
    if (threadIdx.x == 0) {
        status[2] = flags[1];
        status[3] = flags[0];
    }
}

__global__ __launch_bounds__(kScanBlock) void scan_apply_kernel(const int32_t *__restrict__ a,
                                                                const int32_t *__restrict__ b, int64_t n,
                                                                const int64_t *__restrict__ partials, int nblocks,
                                                                int64_t *__restrict__ oa, int64_t *__restrict__ ob) {
    __shared__ int64_t sh[kScanBlock];
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    int32_t va[kScanItems], vb[kScanItems];
    int64_t sa = 0, sb = 0;
    for (int q = 0; q < kScanItems; q++) {
        va[q] = base + q < n ? a[base + q] : 0;
        vb[q] = base + q < n ? b[base + q] : 0;
        sa += va[q];
        sb += vb[q];
    }
    int64_t ta, tb;
    int64_t ea = block_exclusive_scan(sa, sh, ta) + partials[blockIdx.x];
    int64_t eb = block_exclusive_scan(sb, sh, tb) + partials[nblocks + blockIdx.x];
    for (int q = 0; q < kScanItems; q++) {
        if (base + q < n) {
            oa[base + q] = ea;
            ob[base + q] = eb;
        }
        ea += va[q];
        eb += vb[q];
    }
}

hipError_t launch_scan(const bh_grid *g, const bh_moments *m, bh_lists *L, hipStream_t s) {
    const int64_t n = g->n_groups;
    const int nblocks = (int)((n + kScanTile - 1) / kScanTile);
    hipLaunchKernelGGL(scan_reduce_kernel, dim3(nblocks), dim3(kScanBlock), 0, s, L->d_far_cnt, L->d_near_cnt, n,
                       L->d_partials, nblocks);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(scan_partials_kernel, dim3(1), dim3(kScanBlock), 0, s, L->d_partials, nblocks,
                       L->d_far_off + n, L->d_near_off + n, m->d_flags, L->d_status);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(scan_apply_kernel, dim3(nblocks), dim3(kScanBlock), 0, s, L->d_far_cnt, L->d_near_cnt, n,
                       L->d_partials, nblocks, L->d_far_off, L->d_near_off);
    return hipGetLastError();
}

// ---------------------------------------------------------------- pair sums

// 1/sqrt(x) in fp64: hardware estimate refined by two Newton steps
// y <- y (3 - x y^2) / 2, each step roughly doubling the correct bits.
__device__ __forceinline__ double rsqrt64(double x) {
    double y = __builtin_amdgcn_rsq(x);
    double h = 0.5 * x;
    y = y * fma(-h * y, y, 1.5);
    y = y * fma(-h * y, y, 1.5);
    return y;
}

// fp32 far term of one node for one cell, added to `part`:
//   M/d + R^T Q R / (2 d^5) = (M + qd / d^4) / d,  qd = R^T (Q/2) R,
// with the node record p = (X, Y, Z, M), q = (Qxx/2, Qyy/2, Qzz/2, Qxy),
// u = (Qxz, Qyz, -, -).  v_rsq_f32 is used bare: d^2 >= (h/2)^2 is far from
// the denormal range, so the library guard around it is not needed.
__device__ __forceinline__ float far_term(float px, float py, float pz, const float4 p, const float4 q,
                                          const float4 u, float part) {
    const float dx = px - p.x, dy = py - p.y, dz = pz - p.z;
    const float x2 = dx * dx, y2 = dy * dy, z2 = dz * dz;
    const float r2 = (x2 + y2) + z2;
    const float ri = __builtin_amdgcn_rsqf(r2);
    float qd = q.x * x2;
    qd = fmaf(q.y, y2, qd);
    qd = fmaf(q.z, z2, qd);
    float t = q.w * dy;
    t = fmaf(u.x, dz, t);
    qd = fmaf(t, dx, qd);
    qd = fmaf(u.y * dy, dz, qd);
    const float ri2 = ri * ri;
    t = qd * ri2;
    t = fmaf(t, ri2, p.w);
    return fmaf(t, ri, part);
}

// fp64 far term; the record is the fp64 moments row:
// p = (X, Y, Z, M), q = (Qxx, Qyy, Qzz, Qxy), u = (Qxz, Qyz, delta, -).
__device__ __forceinline__ double far_term(double px, double py, double pz, const double4 p, const double4 q,
                                           const double4 u, double part) {
    const double dx = px - p.x, dy = py - p.y, dz = pz - p.z;
    const double r2 = dx * dx + dy * dy + dz * dz;
    const double ri = rsqrt64(r2);
    const double ri2 = ri * ri;
    const double quad = 0.5 * (q.x * dx * dx + q.y * dy * dy + q.z * dz * dz) +
                        (q.w * dx * dy + u.x * dx * dz + u.y * dy * dz);
    return part + (p.w * ri + quad * (ri2 * ri2 * ri));
}

// monopole only: M / d
__device__ __forceinline__ float far_monopole(float px, float py, float pz, const float4 p, float part) {
    const float dx = px - p.x, dy = py - p.y, dz = pz - p.z;
    const float r2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
    return fmaf(p.w, __builtin_amdgcn_rsqf(r2), part);
}
__device__ __forceinline__ double far_monopole(double px, double py, double pz, const double4 p, double part) {
    const double dx = px - p.x, dy = py - p.y, dz = pz - p.z;
    const double r2 = dx * dx + dy * dy + dz * dz;
    return part + p.w * rsqrt64(r2);
}

__device__ __forceinline__ float near_pair(float px, float py, float pz, const float4 s, float part) {
    const float dx = px - s.x, dy = py - s.y, dz = pz - s.z;
    const float r2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
    return fmaf(s.w, __builtin_amdgcn_rsqf(r2), part);
}
__device__ __forceinline__ float near_pair_self(float px, float py, float pz, const float4 s, float part) {
    const float dx = px - s.x, dy = py - s.y, dz = pz - s.z;
    const float r2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
    const float ri = __builtin_amdgcn_rsqf(r2);
    return fmaf(r2 > 0.f ? s.w : 0.f, r2 > 0.f ? ri : 0.f, part);
}
__device__ __forceinline__ double near_pair(double px, double py, double pz, const double4 s, double part) {
    const double dx = px - s.x, dy = py - s.y, dz = pz - s.z;
    const double r2 = dx * dx + dy * dy + dz * dz;
    return part + s.w * rsqrt64(r2);
}
__device__ __forceinline__ double near_pair_self(double px, double py, double pz, const double4 s, double part) {
    const double dx = px - s.x, dy = py - s.y, dz = pz - s.z;
    const double r2 = dx * dx + dy * dy + dz * dz;
    return r2 > 0.0 ? part + s.w * rsqrt64(r2) : part;
}

__device__ __forceinline__ float rsq_any(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double rsq_any(double x) { return rsqrt64(x); }

// Potential and acceleration of one far node (monopole + quadrupole) at one
// cell: the gradient of the far term taken term by term.  The staged record
// holds the full Q: p = (X, Y, Z, M), q = (Qxx, Qyy, Qzz, Qxy), u = (Qxz, Qyz,
// -, -).  Accumulates the bracket of phi = -G [M/d + R^T Q R / (2 d^5)] into
// phi and of g = G [Q R / d^5 - (M / d^3 + 5/2 R^T Q R / d^7) R] into g.
template <typename real, typename V4>
__device__ __forceinline__ void far_term_acc(real px, real py, real pz, const V4 p, const V4 q, const V4 u, real &phi,
                                             real &gx, real &gy, real &gz) {
    const real dx = px - p.x, dy = py - p.y, dz = pz - p.z;
    const real r2 = dx * dx + dy * dy + dz * dz;
    const real ri = rsq_any(r2);
    const real ri2 = ri * ri;
    const real qx = q.x * dx + q.w * dy + u.x * dz;
    const real qy = q.w * dx + q.y * dy + u.y * dz;
    const real qz = u.x * dx + u.y * dy + q.z * dz;
    const real rqr = dx * qx + dy * qy + dz * qz;
    const real ri3 = ri * ri2;
    const real w5 = ri3 * ri2;
    const real t5 = rqr * w5;
    phi += p.w * ri + (real)0.5 * t5;
    const real s = p.w * ri3 + (real)2.5 * (t5 * ri2);
    gx += w5 * qx - s * dx;
    gy += w5 * qy - s * dy;
    gz += w5 * qz - s * dz;
}

// Potential and acceleration of one near cell (none for the cell itself when
// SELF: a zero distance contributes nothing).
template <typename real, bool SELF, typename V4>
__device__ __forceinline__ void near_pair_acc(real px, real py, real pz, const V4 c, real &phi, real &gx, real &gy,
                                              real &gz) {
    const real dx = px - c.x, dy = py - c.y, dz = pz - c.z;
    const real r2 = dx * dx + dy * dy + dz * dz;
    const real r0 = rsq_any(r2);
    const real ri = SELF ? (r2 > (real)0 ? r0 : (real)0) : r0;  // the cell itself: 1/d -> 0, not inf
    const real mri = c.w * ri;
    const real w = mri * ri * ri;
    phi += mri;
    gx -= w * dx;
    gy -= w * dy;
    gz -= w * dz;
}

// Repacks a staged near tile of n bottom nodes (T[8b + k] = cell k of node
// b, Morton order: bit 0 x, bit 1 y, bit 2 z) into 16 values per node behind
// it, at T + 64: the first cell, the lattice steps along x, y and z, then the
// 8 masses (four 16-byte records per node).  The 8 cells of a bottom node are
// the corners of a cube, so a pair needs only the target's offsets to the
// first cell and to the far corner per axis.
__device__ __forceinline__ void near_lattice_pack(float4 *T, int n) {
    const int lane = threadIdx.x & 63;
    float *P = reinterpret_cast<float *>(T + 64);
    if (lane < 8 * n) {
        const float4 c = T[lane];
        const int b = lane >> 3, k = lane & 7;
        P[16 * b + 6 + k] = c.w;
        if (k == 0) {
            P[16 * b + 0] = c.x;
            P[16 * b + 1] = c.y;
            P[16 * b + 2] = c.z;
            P[16 * b + 3] = T[lane + 1].x - c.x;
            P[16 * b + 4] = T[lane + 2].y - c.y;
            P[16 * b + 5] = T[lane + 4].z - c.z;
        }
    }
    wave_lds_sync();
}

// Sum of m / |x - cell| over the n packed nodes (near_lattice_pack) for the
// lane's cell x: per node the offsets a and a - h to its first cell per axis
// and their squares once, then per cell two adds, the rsqrt and one FMA.
__device__ __forceinline__ float near_lattice_sum(const float4 *P, int n, float mx, float my, float mz) {
    float part = 0.0f;
    for (int b = 0; b < n; b++) {
        const float4 h1 = P[4 * b], h2 = P[4 * b + 1], h3 = P[4 * b + 2], h4 = P[4 * b + 3];
        const float ax = mx - h1.x, ay = my - h1.y, az = mz - h1.z;
        const float bx = ax - h1.w, by = ay - h2.x, bz = az - h2.y;
        const float x0 = ax * ax, x1 = bx * bx, y0 = ay * ay, y1 = by * by, z0 = az * az, z1 = bz * bz;
        const float s00 = x0 + y0, s10 = x1 + y0, s01 = x0 + y1, s11 = x1 + y1;
        part = fmaf(h2.z, __builtin_amdgcn_rsqf(s00 + z0), part);
        part = fmaf(h2.w, __builtin_amdgcn_rsqf(s10 + z0), part);
        part = fmaf(h3.x, __builtin_amdgcn_rsqf(s01 + z0), part);
        part = fmaf(h3.y, __builtin_amdgcn_rsqf(s11 + z0), part);
        part = fmaf(h3.z, __builtin_amdgcn_rsqf(s00 + z1), part);
        part = fmaf(h3.w, __builtin_amdgcn_rsqf(s10 + z1), part);
        part = fmaf(h4.x, __builtin_amdgcn_rsqf(s01 + z1), part);
        part = fmaf(h4.y, __builtin_amdgcn_rsqf(s11 + z1), part);
    }
    return part;
}

// Per-wavefront tile evaluation.  Far tile: up to 64 node records (3 x V4
// each) staged in T by lane, then read back by every lane as broadcasts.
// Near tile: up to 8 bottom nodes = 64 cells.  Each tile is summed in `real`
// and added to an fp64 accumulator (separate for far and near, so that every
// path that forms the same tiles in the same order gives identical bits).
// ORDER 2: monopole + quadrupole far terms; 0: monopole only (the paper's
// own far field, for comparison)
template <typename real, int ORDER = 2>
struct Tiles {
    using V4 = typename Prec<real>::V4;
    V4 *T;
    const V4 *rec;
    const V4 *cells;
    const int32_t *child;
    V4 me;
    int own_lo;
    double acc_far, acc_near;

    __device__ void init() { acc_far = acc_near = 0.0; }

    __device__ void load(int64_t id, V4 &a, V4 &b, V4 &c) const {
        a = rec[3 * id + 0];
        b = rec[3 * id + 1];
        c = rec[3 * id + 2];
    }
    __device__ void put(int lane, const V4 a, const V4 b, const V4 c) {
        T[3 * lane + 0] = a;
        T[3 * lane + 1] = b;
        T[3 * lane + 2] = c;
    }
    __device__ void stage_far(int lane, int n, int id) {
        if (lane < n) put(lane, rec[3 * (int64_t)id + 0], rec[3 * (int64_t)id + 1], rec[3 * (int64_t)id + 2]);
        wave_lds_sync();
    }
    // keep: whether this lane's cell takes the tile (two 32-cell groups on one
    // wavefront: a tile of one group's list is computed by all lanes and kept
    // by that group's lanes)
    __device__ void sum_far(int n, bool keep = true) {
        real part = 0;
        if (ORDER == 0)
            for (int j = 0; j < n; j++) part = far_monopole(me.x, me.y, me.z, T[3 * j], part);
        else
            for (int j = 0; j < n; j++) part = far_term(me.x, me.y, me.z, T[3 * j], T[3 * j + 1], T[3 * j + 2], part);
        if (keep) acc_far += (double)part;
        wave_lds_sync();
    }
    // A full near tile staged by direct-to-LDS loads (fp32 records: 16 bytes
    // per lane, global_load_lds_dwordx4): lane l's cell lands in T[l] without
    // passing through registers, so the loads stay in flight during the next
    // walk step.  near_issue starts them and returns whether the tile holds one
    // of the wavefront's own cells; near_finish waits for them and sums.
    static constexpr bool kNearAsync = sizeof(real) == 4;
    __device__ bool near_issue(int lane, int cid) {
        const bool own = (unsigned)(cid - own_lo) < 64u;
        __builtin_amdgcn_global_load_lds((const void *)(cells + (int64_t)cid + (lane & 7)),
                                         (__attribute__((address_space(3))) void *)T, 16, 0, 0);
        return __ballot(own) != 0;
    }
    __device__ void near_finish(bool any_own) {
        __builtin_amdgcn_s_waitcnt(0);
        wave_lds_sync();
        near_sum(8, any_own, true);
    }
    // up to 8 bottom nodes given by their first cell (internal order); lane l
    // holds that of node l >> 3.  own_lo: the wavefront's first cell, so a tile
    // holding one of its 64 cells takes the self-pair select.
    __device__ void near_tile(int lane, int n, int cid, bool keep = true) {
        bool own = false;
        if (lane < 8 * n) {
            own = (unsigned)(cid - own_lo) < 64u;
            T[lane] = cells[(int64_t)cid + (lane & 7)];
        }
        const bool any_own = __ballot(own) != 0;
        wave_lds_sync();
        near_sum(n, any_own, keep);
    }
    // fp32 tiles that hold none of the wavefront's cells, on the bottom
    // nodes' cell lattice (near_lattice_pack): a lane takes its offsets a and
    // a - h to each node's first cell per axis and their squares once per
    // node, and one sum per pair; the repacked node is read back with four
    // broadcasts instead of eight.
    static constexpr bool kLattice = sizeof(real) == 4;
    __device__ real near_lattice(int n) const {
        if constexpr (kLattice) return near_lattice_sum(T + 64, n, me.x, me.y, me.z);
        return 0;
    }
    __device__ void near_sum(int n, bool any_own, bool keep) {
        real part = 0;
        if (kLattice && !any_own) {
            if constexpr (kLattice) near_lattice_pack(T, n);
            part = near_lattice(n);
        } else if (!any_own) {
            for (int j = 0; j < 8 * n; j++) part = near_pair(me.x, me.y, me.z, T[j], part);
        } else {
            for (int j = 0; j < 8 * n; j++) part = near_pair_self(me.x, me.y, me.z, T[j], part);
        }
        if (keep) acc_near += (double)part;
        wave_lds_sync();
    }
    __device__ void finish(const WalkArgs &a, int64_t cell) const { a.phi[cell] = -a.G * (acc_far + acc_near); }
};

// The same tiles for the acceleration kernels: potential and acceleration per
// pair, each tile summed in `real` and folded into fp64 accumulators.  The
// fp32 far records keep Q/2 on the diagonal; the staged copy gets the full Q.
template <typename real>
struct TilesAcc {
    using V4 = typename Prec<real>::V4;
    static constexpr bool kNearAsync = false;
    V4 *T;
    const V4 *rec;
    const V4 *cells;
    const int32_t *child;
    V4 me;
    int own_lo;
    double phi, gx, gy, gz;

    __device__ void init() { phi = gx = gy = gz = 0.0; }
    __device__ static V4 full_q(const V4 q) {
        if constexpr (sizeof(real) == 4)
            return make_float4(2.0f * q.x, 2.0f * q.y, 2.0f * q.z, q.w);
        else
            return q;
    }
    __device__ void load(int64_t id, V4 &a, V4 &b, V4 &c) const {
        a = rec[3 * id + 0];
        b = rec[3 * id + 1];
        c = rec[3 * id + 2];
    }
    __device__ void put(int lane, const V4 a, const V4 b, const V4 c) {
        T[3 * lane + 0] = a;
        T[3 * lane + 1] = full_q(b);
        T[3 * lane + 2] = c;
    }
    __device__ void stage_far(int lane, int n, int id) {
        if (lane < n) put(lane, rec[3 * (int64_t)id + 0], rec[3 * (int64_t)id + 1], rec[3 * (int64_t)id + 2]);
        wave_lds_sync();
    }
    __device__ void sum_far(int n, bool keep = true) {
        real p = 0, x = 0, y = 0, z = 0;
        for (int j = 0; j < n; j++) far_term_acc<real>(me.x, me.y, me.z, T[3 * j], T[3 * j + 1], T[3 * j + 2], p, x, y, z);
        if (keep) {
            phi += (double)p;
            gx += (double)x;
            gy += (double)y;
            gz += (double)z;
        }
        wave_lds_sync();
    }
    __device__ void near_tile(int lane, int n, int cid, bool keep = true) {
        bool own = false;
        if (lane < 8 * n) {
            own = (unsigned)(cid - own_lo) < 64u;
            T[lane] = cells[(int64_t)cid + (lane & 7)];
        }
        const bool any_own = __ballot(own) != 0;
        wave_lds_sync();
        real p = 0, x = 0, y = 0, z = 0;
        if (sizeof(real) == 4 && !any_own)
            near_lattice_acc(n, p, x, y, z);
        else if (!any_own)
            for (int j = 0; j < 8 * n; j++) near_pair_acc<real, false>(me.x, me.y, me.z, T[j], p, x, y, z);
        else
            for (int j = 0; j < 8 * n; j++) near_pair_acc<real, true>(me.x, me.y, me.z, T[j], p, x, y, z);
        if (keep) {
            phi += (double)p;
            gx += (double)x;
            gy += (double)y;
            gz += (double)z;
        }
        wave_lds_sync();
    }
    // fp32 tiles away from the wavefront's cells, on the bottom nodes' cell
    // lattice as in Tiles (the offsets a and a - h per axis serve the
    // gradient too); the repacked node records sit behind the tile.
    __device__ void near_lattice_acc(int n, real &p, real &x, real &y, real &z) {
        if constexpr (sizeof(real) == 4) near_lattice_pack(T, n);
        const V4 *P = T + 64;
        for (int b = 0; b < n; b++) {
            const V4 h1 = P[4 * b], h2 = P[4 * b + 1], h3 = P[4 * b + 2], h4 = P[4 * b + 3];
            const real ax = me.x - h1.x, ay = me.y - h1.y, az = me.z - h1.z;
            const real d[2][3] = {{ax, ay, az}, {ax - h1.w, ay - h2.x, az - h2.y}};
            const real sq[2][3] = {{d[0][0] * d[0][0], d[0][1] * d[0][1], d[0][2] * d[0][2]},
                                   {d[1][0] * d[1][0], d[1][1] * d[1][1], d[1][2] * d[1][2]}};
            const real m[8] = {h2.z, h2.w, h3.x, h3.y, h3.z, h3.w, h4.x, h4.y};
#pragma unroll
            for (int k = 0; k < 8; k++) {
                const int i = k & 1, j = (k >> 1) & 1, l = k >> 2;
                const real r2 = (sq[i][0] + sq[j][1]) + sq[l][2];
                const real ri = rsq_any(r2);
                const real mri = m[k] * ri;
                const real w = mri * ri * ri;
                p += mri;
                x -= w * d[i][0];
                y -= w * d[j][1];
                z -= w * d[l][2];
            }
        }
    }
    __device__ void finish(const WalkArgs &a, int64_t cell) const {
        if (a.phi) a.phi[cell] = -a.G * phi;
        a.acc[3 * cell + 0] = a.G * gx;
        a.acc[3 * cell + 1] = a.G * gy;
        a.acc[3 * cell + 2] = a.G * gz;
    }
};

// The tiles of the periodic kernels.  Every pair is taken at its nearest
// image (far nodes are staged at the image nearest the group centre, which
// leaves each lane at most one box length to remove).  A far pair adds,
// beside the 1/|R| and quadrupole terms, the smooth part of the periodic
// Green's function from the table, its Hessian against the quadrupole and
// the background curvature against S: M D(R) + Q:H(R) / 6 + 2 pi S / (3 L^3).
// A near pair adds m psi(R) = m (1/|R| + D(R)), the cell itself m D(0).
// The staged far record: (X', M), the quadrupole as in the path's far
// record, and S in the third vector's third slot.
// Sum over the wavefront of an fp32 value, complete in lane 63: butterflies
// within rows of 16 lanes (quad permutations, half-row and row mirrors), then
// the row sums carried across rows by the row broadcasts of lanes 15 and 31.
__device__ __forceinline__ float wave_total_f32(float v) {
    int t;
    t = __builtin_amdgcn_update_dpp(0, __float_as_int(v), 0xB1, 0xF, 0xF, false);
    v += __int_as_float(t);
    t = __builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x4E, 0xF, 0xF, false);
    v += __int_as_float(t);
    t = __builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x141, 0xF, 0xF, false);
    v += __int_as_float(t);
    t = __builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x140, 0xF, 0xF, false);
    v += __int_as_float(t);
    t = __builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x142, 0xA, 0xF, false);
    v += __int_as_float(t);
    t = __builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x143, 0xC, 0xF, false);
    v += __int_as_float(t);
    return v;
}

// Coefficients of the group-centre cubic of the smooth part, in u / L (u the
// cell's offset from the octant centre): 0 the value; 1-3 the gradient x y z;
// 4-9 second derivatives xx yy zz xy xz yz; 10-19 third derivatives in the
// table's order xxx yyy zzz xxy xxz xyy yyz xzz yzz xyz.
constexpr int kLocalCoefs = 20;

// Sum over the 8 lanes 8b..8b+7 of an fp32 value, in every one of them (quad
// permutations, then the half-row mirror).
__device__ __forceinline__ float group8_total_f32(float v) {
    int t;
    t = __builtin_amdgcn_update_dpp(0, __float_as_int(v), 0xB1, 0xF, 0xF, false);
    v += __int_as_float(t);
    t = __builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x4E, 0xF, 0xF, false);
    v += __int_as_float(t);
    t = __builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x141, 0xF, 0xF, false);
    v += __int_as_float(t);
    return v;
}

// The same totals for fp64 values (each half moved by the same DPP pattern).
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_src_f64(double v) {
    const uint64_t u = (uint64_t)__double_as_longlong(v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)u, CTRL, ROWS, 0xF, false);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(u >> 32), CTRL, ROWS, 0xF, false);
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}
__device__ __forceinline__ double group8_total_f64(double v) {
    v += dpp_src_f64<0xB1, 0xF>(v);
    v += dpp_src_f64<0x4E, 0xF>(v);
    v += dpp_src_f64<0x141, 0xF>(v);
    return v;
}
__device__ __forceinline__ double wave_total_f64(double v) {
    v = group8_total_f64(v);
    v += dpp_src_f64<0x140, 0xF>(v);
    v += dpp_src_f64<0x142, 0xA>(v);
    v += dpp_src_f64<0x143, 0xC>(v);
    return v;
}
__device__ __forceinline__ double readlane_f64(double v, int k) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), k);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), k);
    return __hiloint2double(hi, lo);
}
// The total of a lane-group of 8 (node8) or of the wavefront, in every lane that needs it, as a double.
__device__ __forceinline__ double cubic_total(float v, bool node8) {
    return node8 ? (double)group8_total_f32(v)
                 : (double)__int_as_float(__builtin_amdgcn_readlane(__float_as_int(wave_total_f32(v)), 63));
}
__device__ __forceinline__ double cubic_total(double v, bool node8) {
    return node8 ? group8_total_f64(v) : readlane_f64(wave_total_f64(v), 63);
}

__device__ __forceinline__ double local_cubic(const double (&c)[kLocalCoefs], double x, double y, double z) {
    const double xx = x * x, yy = y * y, zz = z * z;
    const double lin = c[0] + (c[1] * x + c[2] * y + c[3] * z);
    const double quad = 0.5 * (c[4] * xx + c[5] * yy + c[6] * zz) + (c[7] * x * y + c[8] * x * z + c[9] * y * z);
    const double cube = (c[10] * xx * x + c[11] * yy * y + c[12] * zz * z) / 6.0 +
                        0.5 * (c[13] * xx * y + c[14] * xx * z + c[15] * x * yy + c[16] * yy * z + c[17] * x * zz +
                               c[18] * y * zz) +
                        c[19] * x * y * z;
    return lin + quad + cube;
}

// LOCAL: the group-centre cubic of the smooth part is compiled in (one group
// per wavefront).
template <typename real, bool LOCAL = false>
struct TilesPeriodic {
    using V4 = typename Prec<real>::V4;
    static constexpr bool kNearAsync = false;
    V4 *T;
    const V4 *rec;
    const V4 *cells;
    const int32_t *child;
    const double *node_s;
    V4 me;
    int own_lo;
    double acc_far, acc_near;
    EwaldView<real> ew;
    const float *near_c;  // series of D L near the origin (fp32 walks), then the radius^2; null: table only
    real cg[3], box, box_inv, bg;
    real dscale, qscale;  // table value -> D, and the Q:H sum -> Q:H / 6 (fp32 rows are scaled by powers of L)
    // group-centre cubic of the smooth part (groups of small enough cells): the coefficients of
    // sum_s [m_s D + Q_s : H / 6 + bg S_s](c + u) in u / L (order of kLocalCoefs), c the octant's centre, summed
    // by each lane over the sources it took, in its own slice of LDS, then over the wavefront once per group.
    // node8: one cubic per bottom node instead (lanes 8b..8b+7 hold the 8 cells of bottom node b of the
    // octant), each about the node's centre and summed over its 8 lanes, each lane taking every 8th source
    bool local, node8;
    real lh;         // node8: h, the offset of a bottom node's centre from the octant's per axis; else 0
    real local_lim;  // a source at |R_a| <= local_lim on every axis has one nearest image for every cell
    V4 *lsum;        // [kLocalCoefs / 4][64] of this wavefront, in the walk's precision

    __device__ void setup(const WalkArgs &a, const LeafInfo &L, int sub) {
#pragma clang fp contract(off)
        const real h = (real)L.h;
        const int i0 = (sub & 1) * 4, j0 = ((sub >> 1) & 1) * 4, k0 = ((sub >> 2) & 1) * 4;
        const real eg = (real)1.5 * h;
        cg[0] = (real)(L.lo[0] + (i0 + 0.5) * L.h) + eg;
        cg[1] = (real)(L.lo[1] + (j0 + 0.5) * L.h) + eg;
        cg[2] = (real)(L.lo[2] + (k0 + 0.5) * L.h) + eg;
        box = (real)a.box;
        box_inv = (real)(1.0 / a.box);
        bg = (real)(2.0 * 3.14159265358979323846 / (3.0 * a.box * a.box * a.box));
        ew.tab = (const real *)a.ewald;
        ew.sp = (real)a.ewald_sp;
        ew.inv_sp = (real)(1.0 / a.ewald_sp);
        ew.n = a.ewald_n;
        ew.inv_box = box_inv;
        ew.sp_box = (real)(a.ewald_sp / a.box);
        // the table gives D L and H L^3; fp32 records hold Q/2 on the diagonal
        dscale = box_inv;
        qscale = (real)(1.0 / ((sizeof(real) == 4 ? 3.0 : 6.0) * a.box * a.box * a.box));
        node_s = a.node_s;
        near_c = sizeof(real) == 4 ? a.ewald_near : nullptr;
        local = false;
        if constexpr (LOCAL) {
            local = L.h <= a.ewald_local_hmax;
            node8 = local && L.h > a.ewald_local_hoct;
            lh = node8 ? h : (real)0;
            local_lim = (real)(0.5 * a.box - 1.5 * L.h - 1e-5 * a.box);
            __shared__ V4 lds_sums[4][kLocalCoefs / 4][64];
            lsum = &lds_sums[threadIdx.x >> 6][0][0];
        }
    }
    __device__ void init() {
        acc_far = acc_near = 0.0;
        if (LOCAL && local) {
            const int lane = __lane_id();
#pragma unroll
            for (int k = 0; k < kLocalCoefs / 4; k++) lsum[64 * k + lane] = V4{0, 0, 0, 0};
        }
    }
    __device__ real image(real x, real c) const { return x - box * rint((x - c) * box_inv); }
    // the centre of this lane's cubic on axis d (cells in Morton order: lane bits 3, 4, 5 place the bottom node)
    __device__ real lcentre(int d) const { return cg[d] + (((__lane_id() >> (3 + d)) & 1) ? lh : -lh); }

    __device__ void load(int64_t id, V4 &a, V4 &b, V4 &c) const {
        a = rec[3 * id + 0];
        b = rec[3 * id + 1];
        c = rec[3 * id + 2];
        if constexpr (sizeof(real) == 8) c.z = node_s[id];  // the fp64 row keeps delta there
    }
    __device__ void put(int lane, V4 a, const V4 b, const V4 c) {
        a.x = image(a.x, cg[0]);
        a.y = image(a.y, cg[1]);
        a.z = image(a.z, cg[2]);
        T[3 * lane + 0] = a;
        T[3 * lane + 1] = b;
        T[3 * lane + 2] = c;
    }
    __device__ void stage_far(int lane, int n, int id) {
        if (lane < n) {
            V4 a, b, c;
            load(id, a, b, c);
            put(lane, a, b, c);
        }
        wave_lds_sync();
    }
    // One source's part of the group-centre cubic, added to c: the source at
    // R = c - X from the cubic's centre, the table's cubic about R's point (the
    // expansion a pair lookup makes) re-expanded about u = 0 and mass
    // weighted; a far node (q, w not null: q = (Qxx/2, Qyy/2, Qzz/2, Qxy),
    // w = (Qxz, Qyz, S, -)) adds its quadrupole's Hessian term, whose Hessian
    // is first order in the offset as in far_eval, and bg S.  Odd powers of a
    // coordinate take the sign of R's coordinate (the table is folded).
    __device__ void local_source(real Rx, real Ry, real Rz, real m, const V4 *q, const V4 *w,
                                 real (&c)[kLocalCoefs]) const {
        const EwaldPoint<real> p = ewald_point(ew, Rx, Ry, Rz);
        real v[kEwaldValues];
        ewald_fetch(ew, p.row, v);
        const real x = p.dx, y = p.dy, z = p.dz;
        const real kxx = v[10] * x + v[13] * y + v[14] * z;
        const real kyy = v[15] * x + v[11] * y + v[16] * z;
        const real kzz = v[17] * x + v[18] * y + v[12] * z;
        const real kxy = v[13] * x + v[15] * y + v[19] * z;
        const real kxz = v[14] * x + v[19] * y + v[17] * z;
        const real kyz = v[19] * x + v[16] * y + v[18] * z;
        const real t3 = (real)1 / (real)3;
        // value D0 + d.(g + (H + K/3) d / 2), gradient g + (H + K/2) d, Hessian H + K (K = T d)
        const real wx = (v[4] + kxx * t3) * x + (v[7] + kxy * t3) * y + (v[8] + kxz * t3) * z;
        const real wy = (v[7] + kxy * t3) * x + (v[5] + kyy * t3) * y + (v[9] + kyz * t3) * z;
        const real wz = (v[8] + kxz * t3) * x + (v[9] + kyz * t3) * y + (v[6] + kzz * t3) * z;
        const real val = v[0] + x * (v[1] + (real)0.5 * wx) + y * (v[2] + (real)0.5 * wy) + z * (v[3] + (real)0.5 * wz);
        const real gx = v[1] + (v[4] + (real)0.5 * kxx) * x + (v[7] + (real)0.5 * kxy) * y + (v[8] + (real)0.5 * kxz) * z;
        const real gy = v[2] + (v[7] + (real)0.5 * kxy) * x + (v[5] + (real)0.5 * kyy) * y + (v[9] + (real)0.5 * kyz) * z;
        const real gz = v[3] + (v[8] + (real)0.5 * kxz) * x + (v[9] + (real)0.5 * kyz) * y + (v[6] + (real)0.5 * kzz) * z;
        const real sx = p.sx, sy = p.sy, sz = p.sz;
        const real hxx = v[4] + kxx, hyy = v[5] + kyy, hzz = v[6] + kzz;
        const real hxy = (v[7] + kxy) * (sx * sy), hxz = (v[8] + kxz) * (sx * sz), hyz = (v[9] + kyz) * (sy * sz);
        const real txxx = sx * v[10], tyyy = sy * v[11], tzzz = sz * v[12], txxy = sy * v[13], txxz = sz * v[14];
        const real txyy = sx * v[15], tyyz = sz * v[16], txzz = sx * v[17], tyzz = sy * v[18];
        const real txyz = (sx * sy * sz) * v[19];
        const real md = m * dscale;
        c[0] += md * val;
        c[1] += md * (sx * gx);
        c[2] += md * (sy * gy);
        c[3] += md * (sz * gz);
        c[4] += md * hxx;
        c[5] += md * hyy;
        c[6] += md * hzz;
        c[7] += md * hxy;
        c[8] += md * hxz;
        c[9] += md * hyz;
        c[10] += md * txxx;
        c[11] += md * tyyy;
        c[12] += md * tzzz;
        c[13] += md * txxy;
        c[14] += md * txxz;
        c[15] += md * txyy;
        c[16] += md * tyyz;
        c[17] += md * txzz;
        c[18] += md * tyzz;
        c[19] += md * txyz;
        if (q) {
            const V4 Q = *q, W = *w;
            // fp32 records hold Q/2 on the diagonal (qscale 1/(3 L^3)), fp64 records Q (qscale 1/(6 L^3))
            const real o = sizeof(real) == 4 ? (real)1 : (real)2;
            const real qs = qscale;
            c[0] += qs * ((Q.x * hxx + Q.y * hyy + Q.z * hzz) + o * (Q.w * hxy + W.x * hxz + W.y * hyz)) + bg * W.z;
            c[1] += qs * ((Q.x * txxx + Q.y * txyy + Q.z * txzz) + o * (Q.w * txxy + W.x * txxz + W.y * txyz));
            c[2] += qs * ((Q.x * txxy + Q.y * tyyy + Q.z * tyzz) + o * (Q.w * txyy + W.x * txyz + W.y * tyyz));
            c[3] += qs * ((Q.x * txxz + Q.y * tyyz + Q.z * tzzz) + o * (Q.w * txyz + W.x * txzz + W.y * tyzz));
        }
    }
    // a lane's coefficients added to its running sums (its own LDS slice: no other lane reads it before finish)
    __device__ void local_add(const real (&c)[kLocalCoefs], int lane) {
#pragma unroll
        for (int k = 0; k < kLocalCoefs / 4; k++) {
            V4 t = lsum[64 * k + lane];
            t.x += c[4 * k];
            t.y += c[4 * k + 1];
            t.z += c[4 * k + 2];
            t.w += c[4 * k + 3];
            lsum[64 * k + lane] = t;
        }
    }
    // whether every staged source (lanes < n, the position in s) is at the same nearest image from all the
    // octant's cells
    __device__ bool local_ok(bool mine, real sx, real sy, real sz) const {
        const bool bad = mine && (fabs(cg[0] - sx) > local_lim || fabs(cg[1] - sy) > local_lim ||
                                  fabs(cg[2] - sz) > local_lim);
        return __ballot(bad) == 0;
    }
    // a far tile of a local group: 1/|R| and the quadrupole pair by pair (the positions staged at the image
    // nearest the octant centre), the smooth part through the cubic
    __device__ void far_local(int n, int lane) {
        const V4 *t = T;
        const V4 m = me;
        real part = 0;
        for (int j = 0; j < n; j++) {
            const V4 p = t[3 * j], q = t[3 * j + 1], w = t[3 * j + 2];
            const real dx = m.x - p.x, dy = m.y - p.y, dz = m.z - p.z;
            const real ri = rsq_any(dx * dx + dy * dy + dz * dz);
            const real ri2 = ri * ri;
            real quad;
            if constexpr (sizeof(real) == 4)  // Q/2 on the diagonal
                quad = (q.x * dx * dx + q.y * dy * dy + q.z * dz * dz) + (q.w * dx * dy + w.x * dx * dz + w.y * dy * dz);
            else
                quad = (real)0.5 * (q.x * dx * dx + q.y * dy * dy + q.z * dz * dz) +
                       (q.w * dx * dy + w.x * dx * dz + w.y * dy * dz);
            part += p.w * ri + quad * (ri2 * ri2 * ri);
        }
        acc_far += (double)part;
        const real c0 = lcentre(0), c1 = lcentre(1), c2 = lcentre(2);
        // the lane's sources: its own node, or (node8) every 8th node from its slot in the bottom node
        const int step = node8 ? 8 : 64;
        real c[kLocalCoefs] = {};
        for (int j = node8 ? (lane & 7) : lane; j < n; j += step) {
            const V4 p = t[3 * j], q = t[3 * j + 1], w = t[3 * j + 2];
            local_source(c0 - p.x, c1 - p.y, c2 - p.z, p.w, &q, &w, c);
        }
        local_add(c, lane);
    }
    // The cell's nearest image R of a staged position and its table point.
    struct Pair {
        real dx, dy, dz;
        EwaldPoint<real> ep;
    };
    __device__ Pair pair_at(const V4 p) const {
        Pair c;
        c.dx = me.x - p.x;
        c.dy = me.y - p.y;
        c.dz = me.z - p.z;
        c.dx -= box * rint(c.dx * box_inv);
        c.dy -= box * rint(c.dy * box_inv);
        c.dz -= box * rint(c.dz * box_inv);
        c.ep = ewald_point(ew, c.dx, c.dy, c.dz);
        return c;
    }
    // sum over j < n of eval(pair, table row, j), the table row of pair j + 1
    // fetched before pair j is evaluated (two register buffers in turn)
    template <typename At, typename Eval>
    __device__ real pipelined(int n, At at, Eval eval) const {
        real part = 0;
        if (n <= 0) return part;
        if constexpr (LOCAL) {  // fallback tiles of this kernel are few: one row at a time, fewer registers held
            real v[kEwaldValues];
            for (int j = 0; j < n; j++) {
                const Pair c = pair_at(at(j));
                ewald_fetch(ew, c.ep.row, v);
                part += eval(c, v, j);
            }
            return part;
        }
        Pair ca = pair_at(at(0)), cb;
        real va[kEwaldValues], vb[kEwaldValues];
        ewald_fetch(ew, ca.ep.row, va);
        for (int j = 0;; j += 2) {
            const bool m1 = j + 1 < n;
            if (m1) {
                cb = pair_at(at(j + 1));
                ewald_fetch(ew, cb.ep.row, vb);
            }
            part += eval(ca, va, j);
            if (!m1) break;
            const bool m2 = j + 2 < n;
            if (m2) {
                ca = pair_at(at(j + 2));
                ewald_fetch(ew, ca.ep.row, va);
            }
            part += eval(cb, vb, j + 1);
            if (!m2) break;
        }
        return part;
    }
    // M (1/|R| + D) + R^T Q R / (2 |R|^5) + Q:H / 6 + bg S of one staged node
    __device__ real far_eval(const Pair &c, const real (&v)[kEwaldValues], const V4 p, const V4 q, const V4 u) const {
        const real dx = c.dx, dy = c.dy, dz = c.dz;
        const real r2 = dx * dx + dy * dy + dz * dz;
        const real ri = rsq_any(r2);
        const real ri2 = ri * ri;
        real H[6];
        const real D = ewald_eval(c.ep, v, H);
        real quad, qh;
        if constexpr (sizeof(real) == 4) {  // q = (Qxx/2, Qyy/2, Qzz/2, Qxy), u = (Qxz, Qyz, S, -)
            quad = (q.x * dx * dx + q.y * dy * dy + q.z * dz * dz) + (q.w * dx * dy + u.x * dx * dz + u.y * dy * dz);
            qh = ((q.x * H[0] + q.y * H[1] + q.z * H[2]) + (q.w * H[3] + u.x * H[4] + u.y * H[5])) * qscale;
        } else {  // q = (Qxx, Qyy, Qzz, Qxy), u = (Qxz, Qyz, S, -)
            quad = (real)0.5 * (q.x * dx * dx + q.y * dy * dy + q.z * dz * dz) +
                   (q.w * dx * dy + u.x * dx * dz + u.y * dy * dz);
            qh = ((q.x * H[0] + q.y * H[1] + q.z * H[2]) + (real)2 * (q.w * H[3] + u.x * H[4] + u.y * H[5])) * qscale;
        }
        return p.w * (ri + D * dscale) + quad * (ri2 * ri2 * ri) + qh + bg * u.z;
    }
    __device__ void sum_far(int n, bool keep = true) {
        if constexpr (LOCAL) {
            if (local) {
                const int lane = __lane_id();
                const V4 p = T[3 * (lane < n ? lane : 0)];
                if (local_ok(lane < n, p.x, p.y, p.z)) {
                    far_local(n, lane);
                    wave_lds_sync();
                    return;
                }
            }
        }
        const V4 *t = T;
        const real part = pipelined(
            n, [t](int j) { return t[3 * j]; },
            [this, t](const Pair &c, const real(&v)[kEwaldValues], int j) {
                return far_eval(c, v, t[3 * j], t[3 * j + 1], t[3 * j + 2]);
            });
        if (keep) acc_far += (double)part;
        wave_lds_sync();
    }
    // up to 8 bottom nodes given by their first cell, lane l holds that of
    // node l >> 3; each cell m (1/|R| + D), the cell itself D(0) only.  In
    // fp32, D comes from the near-origin series while every pair of the tile
    // lies within its radius (the usual case for near cells), else the whole
    // tile is summed again through the table.
    __device__ real near_series(int n, bool &inside) const {
        const real c0 = near_c[0], c1 = near_c[1], c2 = near_c[2], c3 = near_c[3], c4 = near_c[4], c5 = near_c[5];
        const real c6 = near_c[6], c7 = near_c[7], c8 = near_c[8], c9 = near_c[9], c10 = near_c[10];
        const real rad2 = near_c[11];
        real part = 0;
        bool out = false;
        for (int j = 0; j < 8 * n; j++) {
            const V4 s = T[j];
            real dx = me.x - s.x, dy = me.y - s.y, dz = me.z - s.z;
            dx -= box * rint(dx * box_inv);
            dy -= box * rint(dy * box_inv);
            dz -= box * rint(dz * box_inv);
            const real ux = dx * box_inv, uy = dy * box_inv, uz = dz * box_inv;
            const real X = ux * ux, Y = uy * uy, Z = uz * uz;
            const real XY = X * Y;
            const real e1 = (X + Y) + Z, e2 = fmaf(Z, X + Y, XY), e3 = XY * Z;
            out |= e1 > rad2;
            const real a = fmaf(e1, fmaf(e1, fmaf(e1, c7, c4), c2), c1);
            const real b = fmaf(e1, fmaf(e1, c8, c5), fmaf(e2, c9, c3));
            const real dl = fmaf(e1, a, fmaf(e2, b, fmaf(e3, fmaf(e1, c10, c6), c0)));
            const real ri = e1 > (real)0 ? rsq_any(e1) * box_inv : (real)0;
            part = fmaf(s.w, ri + dl * dscale, part);
        }
        inside = __ballot(out) == 0;
        return part;
    }
    __device__ void near_tile(int lane, int n, int cid, bool keep = true) {
        V4 s{};
        if (lane < 8 * n) {
            s = cells[(int64_t)cid + (lane & 7)];
            if (LOCAL && local) {  // at the image nearest the octant centre (pairs below take their own images anyway)
                s.x = image(s.x, cg[0]);
                s.y = image(s.y, cg[1]);
                s.z = image(s.z, cg[2]);
            }
            T[lane] = s;
        }
        wave_lds_sync();
        if constexpr (LOCAL) {
            if (local && local_ok(lane < 8 * n, s.x, s.y, s.z)) {
                // the tile's nodes lie within L/2 - 1.5h of the octant centre, so the 8 cells of a node keep
                // their lattice after the imaging above; in fp32 tiles without the wavefront's own cells are
                // summed on it, the others pair by pair, skipping the self pair
                const bool own = lane < 8 * n && cid >= own_lo && cid < own_lo + 64;
                real part = 0;
                if (sizeof(real) == 4 && __ballot(own) == 0) {
                    if constexpr (sizeof(real) == 4) {
                        near_lattice_pack(T, n);
                        part = near_lattice_sum(T + 64, n, me.x, me.y, me.z);
                    }
                } else {
                    for (int j = 0; j < 8 * n; j++) {
                        const V4 q = T[j];
                        const real dx = me.x - q.x, dy = me.y - q.y, dz = me.z - q.z;
                        const real r2 = dx * dx + dy * dy + dz * dz;
                        part += q.w * (r2 > (real)0 ? rsq_any(r2) : (real)0);
                    }
                }
                acc_near += (double)part;
                const real c0 = lcentre(0), c1 = lcentre(1), c2 = lcentre(2);
                const int step = node8 ? 8 : 64;
                real c[kLocalCoefs] = {};
                for (int j = node8 ? (lane & 7) : lane; j < 8 * n; j += step) {
                    const V4 q = T[j];
                    local_source(c0 - q.x, c1 - q.y, c2 - q.z, q.w, nullptr, nullptr, c);
                }
                local_add(c, lane);
                wave_lds_sync();
                return;
            }
        }
        const V4 *t = T;
        real part = 0;
        bool done = false;
        if (near_c) part = near_series(n, done);
        if (!done)
            part = pipelined(
                8 * n, [t](int j) { return t[j]; },
                [this, t](const Pair &c, const real(&v)[kEwaldValues], int j) {
                    const real r2 = c.dx * c.dx + c.dy * c.dy + c.dz * c.dz;
                    const real ri = r2 > (real)0 ? rsq_any(r2) : (real)0;
                    return t[j].w * (ri + ewald_eval<real>(c.ep, v, nullptr) * dscale);
                });
        if (keep) acc_near += (double)part;
        wave_lds_sync();
    }
    __device__ void finish(const WalkArgs &a, int64_t cell) const {
        double smooth = 0.0;
        if constexpr (LOCAL) {
            if (local) {
                const int lane = __lane_id();
                double c[kLocalCoefs];
#pragma unroll
                for (int k = 0; k < kLocalCoefs / 4; k++) {
                    const V4 t = lsum[64 * k + lane];
                    const real v4[4] = {t.x, t.y, t.z, t.w};
#pragma unroll
                    for (int i = 0; i < 4; i++) c[4 * k + i] = cubic_total(v4[i], node8);
                }
                smooth = local_cubic(c, (double)((me.x - lcentre(0)) * box_inv), (double)((me.y - lcentre(1)) * box_inv),
                                     (double)((me.z - lcentre(2)) * box_inv));
            }
        }
        a.phi[cell] = -a.G * (acc_far + acc_near + smooth);
    }
};

struct PotArgs {
    const int64_t *far_off, *near_off;
    const int32_t *far_idx, *near_idx;
    const void *far_rec;         // FarRec32 (fp32) or fp64 moments (kMom doubles)
    const int32_t *child;        // node -> first internal cell (bottom nodes)
    const void *cells;           // float4 / double4, internal order
    const LeafInfo *leaves;
    int64_t n_items;             // wavefronts: 64-cell octants, or 32-cell groups
    int gcells;
    double G;
    double *phi;
};

__device__ __forceinline__ int64_t phi_index(const LeafInfo &L, int sub, int lane) {
    int i, j, k;
    demorton9(sub * 64 + lane, i, j, k);
    return (int64_t)L.canon * kCellsPerBlock + k * 64 + j * 8 + i;
}

// One wavefront per 64-cell octant of a group of 64 or more cells (the
// octants of one group read the same lists), or per 32-cell group (lanes
// 32-63 idle).  Lane = cell in Morton order.
template <typename real>
__global__ __launch_bounds__(256) void potential_kernel(PotArgs a) {
    using V4 = typename Prec<real>::V4;
    __shared__ V4 tile[4][64 * 3];
    const int w = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    const int64_t q = (int64_t)blockIdx.x * 4 + w;
    if (q >= a.n_items) return;
    int f, sub, cell;
    int64_t g;
    if (a.gcells == 32) {
        g = q;
        f = (int)(q >> 4);
        sub = (int)((q & 15) >> 1);
        cell = (int)(q & 15) * 32 + (lane & 31);
    } else {
        f = (int)(q >> 3);
        sub = (int)(q & 7);
        g = q / (a.gcells >> 6);
        cell = sub * 64 + lane;
    }
    const LeafInfo L = a.leaves[f];
    Tiles<real> S;
    S.T = tile[w];
    S.rec = (const V4 *)a.far_rec;
    S.cells = (const V4 *)a.cells;
    S.child = a.child;
    S.own_lo = f * kCellsPerBlock + sub * 64;
    S.me = S.cells[(int64_t)f * kCellsPerBlock + cell];
    S.init();
    const int64_t fb = a.far_off[g], fe = a.far_off[g + 1];
    for (int64_t b = fb; b < fe; b += 64) {
        const int n = (int)(fe - b < 64 ? fe - b : 64);
        S.stage_far(lane, n, lane < n ? a.far_idx[b + lane] : 0);
        S.sum_far(n);
    }
    const int64_t nb = a.near_off[g], ne = a.near_off[g + 1];
    for (int64_t b = nb; b < ne; b += 8) {
        const int n = (int)(ne - b < 8 ? ne - b : 8);
        S.near_tile(lane, n, lane < 8 * n ? a.child[a.near_idx[b + (lane >> 3)]] : 0);
    }
    if (a.gcells == 32 && lane >= 32) return;
    int i, j, k;
    demorton9(cell, i, j, k);
    a.phi[(int64_t)L.canon * kCellsPerBlock + k * 64 + j * 8 + i] = -a.G * (S.acc_far + S.acc_near);
}

hipError_t launch_potential(const bh_grid *g, const bh_moments *m, const bh_lists *L, double G, int precision,
                            double *phi, hipStream_t s) {
    PotArgs a;
    a.far_off = L->d_far_off;
    a.near_off = L->d_near_off;
    a.far_idx = L->d_far;
    a.near_idx = L->d_near;
    a.child = g->d_child;
    a.leaves = g->d_leaves;
    a.gcells = g->group_cells;
    a.n_items = g->group_cells == 32 ? g->n_groups : g->n_units;
    a.G = G;
    a.phi = phi;
    const int blocks = (int)((a.n_items + 3) / 4);
    if (precision == BH_FP64) {
        a.far_rec = m->d_mom;
        a.cells = m->d_cell64;
        hipLaunchKernelGGL(potential_kernel<double>, dim3(blocks), dim3(256), 0, s, a);
    } else {
        a.far_rec = m->d_f32;
        a.cells = m->d_cell32;
        hipLaunchKernelGGL(potential_kernel<float>, dim3(blocks), dim3(256), 0, s, a);
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------- fused walk + sums

// Walk and sum in one pass, without materialising the lists: accepted nodes
// and near bottom nodes are buffered in LDS in walk order and summed as soon
// as a full tile (64 far nodes / 8 bottom nodes) is available, so the tiles
// are exactly those the list path forms, in the same order.  A full far tile
// is software-pipelined: its node records are loaded into registers before
// the next walk step, whose own node loads then cover that latency, and are
// summed after it.  Launch bounds set the waves per SIMD (and so the register
// budget) that hide the walk's remaining load latency best.
// Kernel variants by register budget: waves per SIMD the compiler must fit
// (256 VGPRs per SIMD lane / waves).  More waves hide more of the walk's load
// latency, fewer leave more registers to the pipelined far tile; the default
// of each precision is the fastest single-grid variant, and batched solves
// may pick another one.
constexpr int kFusedDefaultWaves32 = 8;
constexpr int kFusedDefaultWaves64 = 4;

// LDS of one 4-wavefront workgroup.  GM 2 (two 32-cell groups per
// wavefront) keeps three far and three near buffers per wavefront: entries of
// both groups, of the first only, of the second only.
template <typename real, int GM = 1>
struct FusedSmem {
    using V4 = typename Prec<real>::V4;
    int stack[4][kWalkStackCap];
    int fbuf[4][GM == 2 ? 3 : 1][128];
    int nbuf[4][GM == 2 ? 3 : 1][72];
    V4 tile[4][64 * 3];
};

// The wavefront's unit (a 64-cell octant, leaf-major): slot q of the dispatch
// order (units by decreasing cost of the previous walk, so that the longest
// start first and the end of the launch is filled with short ones), or q
// itself; -1 past the end.
__device__ __forceinline__ int64_t dispatch_unit(const WalkArgs &a, int64_t q) {
    if (q >= a.n_units) return -1;
    const int64_t u = a.order ? (int64_t)a.order[q] : q;
    // the same for every lane: kept in scalar registers, as is all that derives from it
    return (int64_t)(((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(u >> 32)) << 32) |
                     (uint32_t)__builtin_amdgcn_readfirstlane((int)u));
}

// Wavefront of the workgroup, known to the compiler as the same for every lane.
__device__ __forceinline__ int wave_index() { return __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)); }

// algorithmic cost of a wavefront's work from its tile entries: 28 flop x 64
// cells per far node, 11 flop x 512 pairs per near bottom node
__device__ __forceinline__ uint32_t group_cost(int nfar, int nnear) {
    return 28u * 64u * (uint32_t)nfar + 11u * 512u * (uint32_t)nnear;
}

// Moves the entries past the first `used` of a wavefront's buffer to its front.
__device__ __forceinline__ void buffer_shift(int *B, int used, int &cnt, int lane) {
    const int rest = cnt - used;
    const int v = lane < rest ? B[used + lane] : 0;
    wave_lds_sync();
    if (lane < rest) B[lane] = v;
    cnt = rest;
    wave_lds_sync();
}

// Octant u of the grid described by a, on wavefront w of the workgroup: walk
// and sums of the group containing it (GM 1, groups of 64 or more cells) or
// of the two 32-cell groups it holds (GM 2).  TL: the tile evaluator
// (potential, potential and acceleration, periodic).
template <typename real, typename TL = Tiles<real>, int MAC = 0, int GM = 1>
__device__ __forceinline__ void fused_group(const WalkArgs &a, int64_t u, int w, int lane, FusedSmem<real, GM> &sm) {
    using V4 = typename Prec<real>::V4;
    const int f = (int)(u >> 3), sub = (int)(u & 7);
    const LeafInfo L = a.leaves[f];
    const int gpl = groups_per_leaf(a.gcells);
    const int wpg = GM == 2 ? 1 : (a.gcells >> 6);  // wavefronts per group
    const int run = GM == 2 ? 2 * sub : sub / wpg;   // (first) group of the octant within the block
    const int64_t cg0 = (int64_t)L.canon * gpl + run;
    Walker<real, MAC, GM> W;
    W.init(a, L, group_box<real>(L, a.gcells, run), cg0, sm.stack[w], lane);
    TL S;
    S.T = sm.tile[w];
    S.rec = (const V4 *)a.far_rec;
    S.cells = (const V4 *)a.cells;
    S.child = a.child;
    S.own_lo = f * kCellsPerBlock + sub * 64;
    S.me = S.cells[(int64_t)f * kCellsPerBlock + sub * 64 + lane];
    if constexpr (MAC == 2) S.setup(a, L, sub);
    S.init();
    if constexpr (GM == 1) {
        int *FB = sm.fbuf[w][0];
        int *NB = sm.nbuf[w][0];
        int fcnt = 0, ncnt = 0, ftot = 0, ntot = 0;
        bool pending = false;  // a full far tile waits in p0..p2
        bool npending = false, nown = false;  // a full near tile is on its way into the LDS tile
        V4 p0, p1, p2;
        while (W.size > 0) {
            int id, acc, nr, cid;
            W.step(lane, id, acc, nr, cid);
            if constexpr (TL::kNearAsync) {
                if (npending) {  // staged during the step (it uses the tile before the far records do)
                    S.near_finish(nown);
                    npending = false;
                }
            }
            if (pending) {  // loaded before the step: sum it now
                S.put(lane, p0, p1, p2);
                wave_lds_sync();
                S.sum_far(64);
                pending = false;
            }
            const uint64_t mf = __ballot(acc);
            const uint64_t mn = __ballot(nr);
            if (acc) FB[fcnt + lane_prefix(mf)] = id;
            if (nr) NB[ncnt + lane_prefix(mn)] = cid;
            fcnt += __popcll(mf);
            ncnt += __popcll(mn);
            ftot += __popcll(mf);
            ntot += __popcll(mn);
            wave_lds_sync();
            if (fcnt >= 64) {  // issue the loads of the next full tile; summed after the next step
                S.load(FB[lane], p0, p1, p2);
                pending = true;
                buffer_shift(FB, 64, fcnt, lane);
            }
            // near tiles in buffer order: all but the newest full one now, that one staged during the next step
            while (ncnt >= (TL::kNearAsync ? 16 : 8)) {
                S.near_tile(lane, 8, NB[lane >> 3]);
                buffer_shift(NB, 8, ncnt, lane);
            }
            if constexpr (TL::kNearAsync) {
                if (ncnt >= 8 && W.size > 0) {
                    nown = S.near_issue(lane, NB[lane >> 3]);
                    npending = true;
                    buffer_shift(NB, 8, ncnt, lane);
                }
            }
        }
        W.finish(a, lane);
        if constexpr (TL::kNearAsync) {
            if (npending) S.near_finish(nown);
        }
        while (ncnt >= 8) {  // the last full tiles (the walk has ended)
            S.near_tile(lane, 8, NB[lane >> 3]);
            buffer_shift(NB, 8, ncnt, lane);
        }
        if (pending) {
            S.put(lane, p0, p1, p2);
            wave_lds_sync();
            S.sum_far(64);
        }
        if (fcnt >= 64) {  // at most one more full tile can remain
            S.stage_far(lane, 64, FB[lane]);
            S.sum_far(64);
            buffer_shift(FB, 64, fcnt, lane);
        }
        if (fcnt > 0) {
            S.stage_far(lane, fcnt, lane < fcnt ? FB[lane] : 0);
            S.sum_far(fcnt);
        }
        if (ncnt > 0) S.near_tile(lane, ncnt, lane < 8 * ncnt ? NB[lane >> 3] : 0);
        S.finish(a, phi_index(L, sub, lane));
        if (a.counts && lane == 0 && sub % wpg == 0) {  // one wavefront per group reports its counts
            a.counts[2 * cg0 + 0] = ftot;
            a.counts[2 * cg0 + 1] = ntot;
        }
        if (a.cost_out && lane == 0) a.cost_out[u] = group_cost(ftot, ntot);
    } else {
        // category c: 0 = both groups, 1 = lanes 0-31's group only, 2 = lanes 32-63's only
        int fcnt[3] = {0, 0, 0}, ncnt[3] = {0, 0, 0}, ftot[3] = {0, 0, 0}, ntot[3] = {0, 0, 0};
        const bool low = lane < 32;
        while (W.size > 0) {
            int id, acc, nr, cid;
            W.step(lane, id, acc, nr, cid);
#pragma unroll
            for (int c = 0; c < 3; c++) {
                const int code = c == 0 ? 3 : c;
                const uint64_t mf = __ballot(acc == code);
                const uint64_t mn = __ballot(nr == code);
                if (acc == code) sm.fbuf[w][c][fcnt[c] + lane_prefix(mf)] = id;
                if (nr == code) sm.nbuf[w][c][ncnt[c] + lane_prefix(mn)] = cid;
                fcnt[c] += __popcll(mf);
                ncnt[c] += __popcll(mn);
                ftot[c] += __popcll(mf);
                ntot[c] += __popcll(mn);
            }
            wave_lds_sync();
#pragma unroll
            for (int c = 0; c < 3; c++) {
                const bool keep = c == 0 || (c == 1) == low;
                int *FB = sm.fbuf[w][c];
                int *NB = sm.nbuf[w][c];
                if (fcnt[c] >= 64) {
                    S.stage_far(lane, 64, FB[lane]);
                    S.sum_far(64, keep);
                    buffer_shift(FB, 64, fcnt[c], lane);
                }
                while (ncnt[c] >= 8) {
                    S.near_tile(lane, 8, NB[lane >> 3], keep);
                    buffer_shift(NB, 8, ncnt[c], lane);
                }
            }
        }
        W.finish(a, lane);
#pragma unroll
        for (int c = 0; c < 3; c++) {
            const bool keep = c == 0 || (c == 1) == low;
            int *FB = sm.fbuf[w][c];
            int *NB = sm.nbuf[w][c];
            if (fcnt[c] > 0) {
                S.stage_far(lane, fcnt[c], lane < fcnt[c] ? FB[lane] : 0);
                S.sum_far(fcnt[c], keep);
            }
            if (ncnt[c] > 0) S.near_tile(lane, ncnt[c], lane < 8 * ncnt[c] ? NB[lane >> 3] : 0, keep);
        }
        S.finish(a, phi_index(L, sub, lane));
        if (a.counts && lane == 0) {
            a.counts[2 * cg0 + 0] = ftot[0] + ftot[1];
            a.counts[2 * cg0 + 1] = ntot[0] + ntot[1];
            a.counts[2 * cg0 + 2] = ftot[0] + ftot[2];
            a.counts[2 * cg0 + 3] = ntot[0] + ntot[2];
        }
        if (a.cost_out && lane == 0)
            a.cost_out[u] = group_cost(ftot[0] + ftot[1] + ftot[2], ntot[0] + ntot[1] + ntot[2]);
    }
}

// Attach the schedule to a single-grid fused walk: dispatch in the order that
// the last upward pass built (natural order before there is one), and record
// this walk's costs for the next.
static hipError_t attach_schedule(const bh_grid *, const bh_moments *m, WalkArgs &a, hipStream_t) {
    a.cost_out = m->d_cost;
    a.order = m->order_valid ? m->d_order : nullptr;
    m->cost_valid = true;
    return hipSuccess;
}

// Wavefronts of a single-grid fused launch: one per 64-cell octant, four per
// workgroup; GM 2 for 32-cell groups (two per wavefront).
static dim3 fused_blocks(const bh_grid *g) { return dim3((unsigned)((g->n_units + 3) / 4)); }
static int fused_gm(const bh_grid *g) { return g->group_cells == 32 ? 2 : 1; }

template <typename real, int WAVES, int GM>
__global__ __launch_bounds__(256, WAVES) void walk_potential_kernel(WalkArgs a) {
    __shared__ FusedSmem<real, GM> sm;
    const int w = wave_index();
    const int lane = threadIdx.x & 63;
    const int64_t u = dispatch_unit(a, (int64_t)blockIdx.x * 4 + w);
    if (u < 0) return;
    fused_group<real, Tiles<real>, 0, GM>(a, u, w, lane, sm);
}

// The fused walk with another opening test and/or far-field order (the
// paper's own choices, for comparison); otherwise as walk_potential_kernel.
template <typename real, int WAVES, int MAC, int ORDER, int GM>
__global__ __launch_bounds__(256, WAVES) void walk_potential_opts_kernel(WalkArgs a) {
    __shared__ FusedSmem<real, GM> sm;
    const int w = wave_index();
    const int lane = threadIdx.x & 63;
    const int64_t u = dispatch_unit(a, (int64_t)blockIdx.x * 4 + w);
    if (u < 0) return;
    fused_group<real, Tiles<real, ORDER>, MAC, GM>(a, u, w, lane, sm);
}

hipError_t launch_walk_potential_opts(const bh_grid *g, const bh_moments *m, double theta, const float *theta_group,
                                      int precision, double G, double *phi, int32_t *counts, int mac, int order,
                                      hipStream_t s) {
    if (mac == BH_MAC_CELLS && order == 2)
        return launch_walk_potential(g, m, theta, theta_group, precision, G, phi, counts, s);
    WalkArgs a = fused_args(g, m, theta, theta_group, precision, G, phi, counts, m->walk_epoch);
    hipError_t e0 = attach_schedule(g, m, a, s);
    if (e0 != hipSuccess) return e0;
    const dim3 grid = fused_blocks(g), block(256);
#define BH_OPTS(T, W, M, O)                                                                          \
    do {                                                                                             \
        if (fused_gm(g) == 2)                                                                        \
            hipLaunchKernelGGL((walk_potential_opts_kernel<T, W, M, O, 2>), grid, block, 0, s, a); \
        else                                                                                         \
            hipLaunchKernelGGL((walk_potential_opts_kernel<T, W, M, O, 1>), grid, block, 0, s, a); \
    } while (0)
    if (precision == BH_FP64) {
        if (mac == BH_MAC_GROUP_BOX && order == 2) BH_OPTS(double, kFusedDefaultWaves64, 1, 2);
        else if (mac == BH_MAC_GROUP_BOX) BH_OPTS(double, kFusedDefaultWaves64, 1, 0);
        else BH_OPTS(double, kFusedDefaultWaves64, 0, 0);
    } else {
        if (mac == BH_MAC_GROUP_BOX && order == 2) BH_OPTS(float, kFusedDefaultWaves32, 1, 2);
        else if (mac == BH_MAC_GROUP_BOX) BH_OPTS(float, kFusedDefaultWaves32, 1, 0);
        else BH_OPTS(float, kFusedDefaultWaves32, 0, 0);
    }
#undef BH_OPTS
    return hipGetLastError();
}

// Periodic box (appendix "Periodic boundaries"): the walk with nearest images
// (MAC mode 2), the sums through the periodic Green's function table
// (TilesPeriodic).
constexpr int kPeriodicWaves32 = 4, kPeriodicWaves64 = 2, kPeriodicWavesCubic = 4;
template <typename real, int WAVES, int GM, bool LOCAL = false>
__global__ __launch_bounds__(256, WAVES) void walk_potential_periodic_kernel(WalkArgs a) {
    __shared__ FusedSmem<real, GM> sm;
    const int w = wave_index();
    const int lane = threadIdx.x & 63;
    const int64_t u = dispatch_unit(a, (int64_t)blockIdx.x * 4 + w);
    if (u < 0) return;
    fused_group<real, TilesPeriodic<real, LOCAL>, 2, GM>(a, u, w, lane, sm);
}

void periodic_args(WalkArgs &a, const bh_grid *g, const bh_moments *m, const bh_ewald *e, int precision) {
    a.box = g->topo.box;
    a.ewald = precision == BH_FP64 ? (const void *)e->d_t64c : (const void *)e->d_t32;
    a.ewald_near = precision == BH_FP32 && e->near_radius > 0.0 ? e->d_near : nullptr;
    const bool cubic = g->group_cells >= 64;
    a.ewald_local_hmax = cubic ? ewald_local_hmax(e, kLocalSpreadNode) : 0.0;
    a.ewald_local_hoct = cubic ? ewald_local_hmax(e, kLocalSpreadOctant) : 0.0;
    a.ewald_sp = e->sp;
    a.ewald_n = e->n;
    a.node_s = m->d_s;
}

hipError_t launch_walk_potential_periodic(const bh_grid *g, const bh_moments *m, const bh_ewald *e, double theta,
                                          const float *theta_group, int precision, double G, double *phi,
                                          int32_t *counts, hipStream_t s) {
    WalkArgs a = fused_args(g, m, theta, theta_group, precision, G, phi, counts, m->walk_epoch);
    periodic_args(a, g, m, e, precision);
    hipError_t e0 = attach_schedule(g, m, a, s);
    if (e0 != hipSuccess) return e0;
    const dim3 grid = fused_blocks(g), block(256);
    if (precision == BH_FP64) {
        if (fused_gm(g) == 2)
            hipLaunchKernelGGL((walk_potential_periodic_kernel<double, kPeriodicWaves64, 2>), grid, block, 0, s, a);
        else if (a.ewald_local_hmax > 0.0)
            hipLaunchKernelGGL((walk_potential_periodic_kernel<double, kPeriodicWaves64, 1, true>), grid, block, 0, s,
                               a);
        else
            hipLaunchKernelGGL((walk_potential_periodic_kernel<double, kPeriodicWaves64, 1>), grid, block, 0, s, a);
    } else {
        // groups summing D through the group-centre cubic only in the kernel compiled for it
        if (fused_gm(g) == 2)
            hipLaunchKernelGGL((walk_potential_periodic_kernel<float, kPeriodicWaves32, 2>), grid, block, 0, s, a);
        else if (a.ewald_local_hmax > 0.0)
            hipLaunchKernelGGL((walk_potential_periodic_kernel<float, kPeriodicWavesCubic, 1, true>), grid, block, 0,
                               s, a);
        else
            hipLaunchKernelGGL((walk_potential_periodic_kernel<float, kPeriodicWaves32, 1>), grid, block, 0, s, a);
    }
    return hipGetLastError();
}

// walk_potential_kernel with each group's theta read from an array (the
// learned-theta step's walk, after the inference kernel): a kernel of its own
// name, so that profiles tell per-group-theta walks from fixed-theta ones.
template <typename real, int WAVES, int GM>
__global__ __launch_bounds__(256, WAVES) void walk_potential_theta_kernel(WalkArgs a) {
    __shared__ FusedSmem<real, GM> sm;
    const int w = wave_index();
    const int lane = threadIdx.x & 63;
    const int64_t u = dispatch_unit(a, (int64_t)blockIdx.x * 4 + w);
    if (u < 0) return;
    fused_group<real, Tiles<real>, 0, GM>(a, u, w, lane, sm);
}

hipError_t launch_walk_potential_theta(const bh_grid *g, const bh_moments *m, const float *theta_group,
                                       int precision, double G, double *phi, int32_t *counts, hipStream_t s) {
    WalkArgs a = fused_args(g, m, 1.0, theta_group, precision, G, phi, counts, m->walk_epoch);
    hipError_t e0 = attach_schedule(g, m, a, s);
    if (e0 != hipSuccess) return e0;
    const dim3 grid = fused_blocks(g), block(256);
    if (precision == BH_FP64) {
        if (fused_gm(g) == 2)
            hipLaunchKernelGGL((walk_potential_theta_kernel<double, kFusedDefaultWaves64, 2>), grid, block, 0, s, a);
        else
            hipLaunchKernelGGL((walk_potential_theta_kernel<double, kFusedDefaultWaves64, 1>), grid, block, 0, s, a);
    } else {
        if (fused_gm(g) == 2)
            hipLaunchKernelGGL((walk_potential_theta_kernel<float, kFusedDefaultWaves32, 2>), grid, block, 0, s, a);
        else
            hipLaunchKernelGGL((walk_potential_theta_kernel<float, kFusedDefaultWaves32, 1>), grid, block, 0, s, a);
    }
    return hipGetLastError();
}

// Walk fused with the potential and acceleration sums.  More live values than
// the potential kernel, hence a smaller register budget per wave.
constexpr int kAccelWaves32 = 6;
constexpr int kAccelWaves64 = 4;
template <typename real, int WAVES, int GM>
__global__ __launch_bounds__(256, WAVES) void walk_accel_kernel(WalkArgs a) {
    __shared__ FusedSmem<real, GM> sm;
    const int w = wave_index();
    const int lane = threadIdx.x & 63;
    const int64_t u = dispatch_unit(a, (int64_t)blockIdx.x * 4 + w);
    if (u < 0) return;
    fused_group<real, TilesAcc<real>, 0, GM>(a, u, w, lane, sm);
}

hipError_t launch_walk_accel(const bh_grid *g, const bh_moments *m, double theta, const float *theta_group,
                             int precision, double G, double *phi, double *acc, int32_t *counts, hipStream_t s) {
    WalkArgs a = fused_args(g, m, theta, theta_group, precision, G, phi, counts, m->walk_epoch);
    a.acc = acc;
    hipError_t e0 = attach_schedule(g, m, a, s);
    if (e0 != hipSuccess) return e0;
    const dim3 grid = fused_blocks(g), block(256);
    if (precision == BH_FP64) {
        if (fused_gm(g) == 2)
            hipLaunchKernelGGL((walk_accel_kernel<double, kAccelWaves64, 2>), grid, block, 0, s, a);
        else
            hipLaunchKernelGGL((walk_accel_kernel<double, kAccelWaves64, 1>), grid, block, 0, s, a);
    } else {
        if (fused_gm(g) == 2)
            hipLaunchKernelGGL((walk_accel_kernel<float, kAccelWaves32, 2>), grid, block, 0, s, a);
        else
            hipLaunchKernelGGL((walk_accel_kernel<float, kAccelWaves32, 1>), grid, block, 0, s, a);
    }
    return hipGetLastError();
}

// Many grids in one persistent launch: every wavefront takes the next
// (grid, group) item of `order` from an atomic counter until the queue is
// empty, so uneven grids and groups balance themselves; with `order` sorted
// by decreasing cost the longest groups start first.  Every wave exits once
// the counter passes `total`.
template <typename real, typename TL, int MAC>
__device__ __forceinline__ void batch_queue(const WalkArgs *__restrict__ grids, const int2 *__restrict__ order,
                                            int64_t total, unsigned long long *__restrict__ counter,
                                            FusedSmem<real, 1> &sm) {
    const int w = wave_index();
    const int lane = threadIdx.x & 63;
    while (true) {
        unsigned long long q = 0;
        if (lane == 0) q = atomicAdd(counter, 1ull);
        // lane 0's item, read as a wave-uniform value: the item and its grid's
        // arguments then live in scalar registers, not in 64 copies
        const uint32_t qlo = __builtin_amdgcn_readfirstlane((uint32_t)q);
        const uint32_t qhi = __builtin_amdgcn_readfirstlane((uint32_t)(q >> 32));
        q = ((unsigned long long)qhi << 32) | qlo;
        if (q >= (unsigned long long)total) break;
        const int2 item = order[q];
        fused_group<real, TL, MAC, 1>(grids[item.x], item.y, w, lane, sm);
    }
}

template <typename real, int WAVES>
__global__ __launch_bounds__(256, WAVES) void batch_walk_potential_kernel(
    const WalkArgs *__restrict__ grids, const int2 *__restrict__ order, int64_t total,
    unsigned long long *__restrict__ counter) {
    __shared__ FusedSmem<real, 1> sm;
    batch_queue<real, Tiles<real>, 0>(grids, order, total, counter, sm);
}

// The same queue over grids in one periodic box (nearest-image walk, the
// periodic sums of TilesPeriodic; LOCAL: the group-centre cubics compiled in).
template <typename real, int WAVES, bool LOCAL>
__global__ __launch_bounds__(256, WAVES) void batch_walk_potential_periodic_kernel(
    const WalkArgs *__restrict__ grids, const int2 *__restrict__ order, int64_t total,
    unsigned long long *__restrict__ counter) {
    __shared__ FusedSmem<real, 1> sm;
    batch_queue<real, TilesPeriodic<real, LOCAL>, 2>(grids, order, total, counter, sm);
}

// Clears the queue counter and the device flags of every grid in a batch
// (a kernel rather than a memset, so that the sequence can be captured).
__global__ void batch_reset_kernel(const WalkArgs *__restrict__ grids, int n, unsigned long long *counter) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) *counter = 0ull;
    if (i < n) {
        grids[i].flags[0] = 0;
        grids[i].flags[1] = 0;
    }
}

hipError_t launch_walk_potential(const bh_grid *g, const bh_moments *m, double theta, const float *theta_group,
                                 int precision, double G, double *phi, int32_t *counts, hipStream_t s) {
    if (theta_group) return launch_walk_potential_theta(g, m, theta_group, precision, G, phi, counts, s);
    WalkArgs a = fused_args(g, m, theta, theta_group, precision, G, phi, counts, m->walk_epoch);
    hipError_t e0 = attach_schedule(g, m, a, s);
    if (e0 != hipSuccess) return e0;
    const dim3 grid = fused_blocks(g), block(256);
    if (precision == BH_FP64) {
        if (fused_gm(g) == 2)
            hipLaunchKernelGGL((walk_potential_kernel<double, kFusedDefaultWaves64, 2>), grid, block, 0, s, a);
        else
            hipLaunchKernelGGL((walk_potential_kernel<double, kFusedDefaultWaves64, 1>), grid, block, 0, s, a);
    } else {
        if (fused_gm(g) == 2)
            hipLaunchKernelGGL((walk_potential_kernel<float, kFusedDefaultWaves32, 2>), grid, block, 0, s, a);
        else
            hipLaunchKernelGGL((walk_potential_kernel<float, kFusedDefaultWaves32, 1>), grid, block, 0, s, a);
    }
    return hipGetLastError();
}

WalkArgs fused_args(const bh_grid *g, const bh_moments *m, double theta, const float *theta_group, int precision,
                    double G, double *phi, int32_t *counts, int epoch) {
    WalkArgs a = walk_args(g, m, theta, theta_group, precision, epoch);
    a.far_rec = precision == BH_FP64 ? (const void *)m->d_mom : (const void *)m->d_f32;
    a.cells = precision == BH_FP64 ? (const void *)m->d_cell64 : (const void *)m->d_cell32;
    a.G = G;
    a.phi = phi;
    a.counts = counts;
    return a;
}

hipError_t launch_batch_reset(const WalkArgs *grids, int n, unsigned long long *counter, hipStream_t s) {
    hipLaunchKernelGGL(batch_reset_kernel, dim3((n + 63) / 64), dim3(64), 0, s, grids, n, counter);
    return hipGetLastError();
}

hipError_t launch_batch_walk_potential(const WalkArgs *grids, const int2 *order, int64_t total,
                                       unsigned long long *counter, int precision, int waves, int workgroups,
                                       hipStream_t s) {
    const dim3 grid(workgroups), block(256);
#define BH_BATCH_LAUNCH(T, W) \
    hipLaunchKernelGGL((batch_walk_potential_kernel<T, W>), grid, block, 0, s, grids, order, total, counter)
    if (precision == BH_FP64) {
        switch (waves) {
            case 2: BH_BATCH_LAUNCH(double, 2); break;
            case 4: BH_BATCH_LAUNCH(double, 4); break;
            default: return hipErrorInvalidValue;
        }
    } else {
        switch (waves) {
            case 4: BH_BATCH_LAUNCH(float, 4); break;
            case 6: BH_BATCH_LAUNCH(float, 6); break;
            case 8: BH_BATCH_LAUNCH(float, 8); break;
            default: return hipErrorInvalidValue;
        }
    }
#undef BH_BATCH_LAUNCH
    return hipGetLastError();
}

int fused_waves_per_simd(int precision) { return precision == BH_FP64 ? kFusedDefaultWaves64 : kFusedDefaultWaves32; }

int periodic_waves_per_simd(int precision, bool local) {
    return precision == BH_FP64 ? kPeriodicWaves64 : (local ? kPeriodicWavesCubic : kPeriodicWaves32);
}

hipError_t launch_batch_walk_potential_periodic(const WalkArgs *grids, const int2 *order, int64_t total,
                                                unsigned long long *counter, int precision, bool local,
                                                int workgroups, hipStream_t s) {
    const dim3 grid(workgroups), block(256);
#define BH_BATCH_PERIODIC(T, W, LOC)                                                                         \
    hipLaunchKernelGGL((batch_walk_potential_periodic_kernel<T, W, LOC>), grid, block, 0, s, grids, order, total, \
                       counter)
    if (precision == BH_FP64) {
        if (local)
            BH_BATCH_PERIODIC(double, kPeriodicWaves64, true);
        else
            BH_BATCH_PERIODIC(double, kPeriodicWaves64, false);
    } else {
        if (local)
            BH_BATCH_PERIODIC(float, kPeriodicWavesCubic, true);
        else
            BH_BATCH_PERIODIC(float, kPeriodicWaves32, false);
    }
#undef BH_BATCH_PERIODIC
    return hipGetLastError();
}

bool fused_variant_exists(int precision, int waves) {
    return precision == BH_FP64 ? (waves == 2 || waves == 4) : (waves == 4 || waves == 6 || waves == 8);
}

// ---------------------------------------------------------------- direct

// ACC: out[3 t + k] = -G sum_{j != i} m_j (r_i - r_j)_k / |r_i - r_j|^3
// (acceleration) instead of the potential.
template <bool ACC>
__global__ __launch_bounds__(256) void direct_kernel(const int64_t *__restrict__ targets, int64_t n,
                                                     const double4 *__restrict__ cells, int64_t ncells,
                                                     const int32_t *__restrict__ internal_of_canon, double G,
                                                     double *__restrict__ phi) {
    __shared__ double4 tile[256];
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const bool valid = t < n;
    int64_t self = -1;
    bool ok = false;
    double4 me = make_double4(0, 0, 0, 0);
    if (valid) {
        const int64_t cid = targets[t];
        if (cid >= 0 && cid < ncells) {
            const int64_t leaf = cid / kCellsPerBlock;
            const int local = (int)(cid % kCellsPerBlock);
            const int f = internal_of_canon[leaf];
            self = (int64_t)f * kCellsPerBlock + morton9(local & 7, (local >> 3) & 7, local >> 6);
            me = cells[self];
            ok = true;
        }
    }
    double acc = 0.0, ax = 0.0, ay = 0.0, az = 0.0;
    for (int64_t base = 0; base < ncells; base += 256) {
        __syncthreads();
        tile[threadIdx.x] = cells[base + threadIdx.x];  // ncells is a multiple of 512
        __syncthreads();
        double part = 0.0, px = 0.0, py = 0.0, pz = 0.0;
        for (int j = 0; j < 256; j++) {
            const double4 s = tile[j];
            const double dx = me.x - s.x, dy = me.y - s.y, dz = me.z - s.z;
            const double r2 = dx * dx + dy * dy + dz * dz;
            if (base + j == self) continue;
            if (ACC) {
                const double w = s.w / (r2 * sqrt(r2));
                px -= w * dx;
                py -= w * dy;
                pz -= w * dz;
            } else {
                part += s.w / sqrt(r2);
            }
        }
        acc += part;
        ax += px;
        ay += py;
        az += pz;
    }
    if (!valid) return;
    if (ACC) {
        phi[3 * t + 0] = ok ? G * ax : __builtin_nan("");
        phi[3 * t + 1] = ok ? G * ay : __builtin_nan("");
        phi[3 * t + 2] = ok ? G * az : __builtin_nan("");
    } else {
        phi[t] = ok ? -G * acc : __builtin_nan("");
    }
}

hipError_t launch_direct(const bh_grid *g, const bh_moments *m, const int64_t *targets, int64_t n, double G,
                         double *out, bool accel, hipStream_t s) {
    if (n == 0) return hipSuccess;
    const int blocks = (int)((n + 255) / 256);
    if (accel)
        hipLaunchKernelGGL(direct_kernel<true>, dim3(blocks), dim3(256), 0, s, targets, n, m->d_cell64, g->n_cells,
                           g->d_internal_of_canon, G, out);
    else
        hipLaunchKernelGGL(direct_kernel<false>, dim3(blocks), dim3(256), 0, s, targets, n, m->d_cell64, g->n_cells,
                           g->d_internal_of_canon, G, out);
    return hipGetLastError();
}

}  // namespace bh
