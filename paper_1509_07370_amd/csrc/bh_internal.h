// Internal declarations of the Barnes-Hut library (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <string>
#include <vector>

#include "bh.h"

namespace bh {

constexpr int kNB = 8;          // cells per block edge
constexpr int kCellsPerBlock = 512;
constexpr int kGroupCells = 64;  // cells per group = lanes per wavefront
constexpr int kWalkStackCap = 256;  // LDS stack entries per wavefront (sibling sets)
constexpr int kMaxDepth = 18;

enum NodeFlags : int { FLAG_BOTTOM = 1, FLAG_EMPTY = 2 };

// Walk record, fp32: centre of mass, delta, edge, first child (node id for
// internal nodes, first internal cell id for bottom nodes), flags.  32 bytes.
struct alignas(16) WalkRec32 {
    float x, y, z, delta;
    float l;
    int child;
    int flags;
    int pad;
};
// Walk record, fp64.  48 bytes.
struct alignas(16) WalkRec64 {
    double x, y, z, delta;
    double l;
    int child;
    int flags;
};
// Far-field record, fp32: COM, mass and the quadrupole pre-scaled for
// R^T Q R / 2 = a x^2 + b y^2 + f z^2 + c xy + d xz + e yz
// (a = Qxx/2, b = Qyy/2, f = Qzz/2, c = Qxy, d = Qxz, e = Qyz).  48 bytes.
struct alignas(16) FarRec32 {
    float x, y, z, m;
    float a, b, f, c;
    float d, e, s, pad1;  // s = sum m |r - X|^2 (periodic sums)
};
// fp64 node moments, 12 doubles per node:
//   0 X, 1 Y, 2 Z, 3 M, 4 Qxx, 5 Qyy, 6 Qzz, 7 Qxy, 8 Qxz, 9 Qyz, 10 delta,
//   11 largest single-cell mass below the node (in-block nodes; 0 elsewhere)
constexpr int kMom = 12;

// Per leaf block, internal (Morton) order.  48 bytes.
struct alignas(16) LeafInfo {
    double lo[3];
    double h;         // cell edge
    int canon;        // leaf ordinal in the caller's block list
    int block_node;   // node id of the block
    int oct_first;    // node id of octant 0 (8 consecutive)
    int bot_first;    // node id of bottom node 0 (64 consecutive, Morton order)
};

// Arguments of one grid's walk (and of its fused walk + sums); also the
// per-grid record of a batch, read by the persistent batch kernel.
struct WalkArgs {
    const void *nodes;
    const LeafInfo *leaves;
    const float *theta_group;
    double theta;
    int64_t n_groups;  // groups of gcells cells
    int gcells;        // cells per group: 32, 64, 128, 256 or 512
    int64_t n_units;   // 64-cell octants (8 per leaf block): the fused kernels' wavefronts
    int root;
    int k8_threshold;
    int epoch;
    int *flags;  // flags[1] <- epoch on stack overflow
    // list mode
    int32_t *far_cnt, *near_cnt;
    const int64_t *far_off, *near_off;
    int32_t *far_out, *near_out;
    // fused mode
    const void *far_rec;
    const int32_t *child;
    const void *cells;
    double G;
    double *phi;
    int32_t *counts;
    double *acc;  // accelerations [cell][3] (acceleration kernels only)
    // single-grid fused kernels: dispatch order of the groups (NULL: natural)
    // and each group's algorithmic cost, written for the next call's order
    const int32_t *order;
    uint32_t *cost_out;
    // periodic kernels: box side, the Green's function table (fp32 or fp64 to
    // match the path) and its spacing, and the fp64 S of every node
    double box;
    const void *ewald;
    double ewald_sp;
    int ewald_n;
    const float *ewald_near;  // near-origin series of D (fp32 periodic walks), or null
    double ewald_local_hmax;  // periodic walks: groups of cells no larger sum D through cubics about the
                              // centres of their bottom nodes (0: never)
    double ewald_local_hoct;  // ... and no larger than this, through one cubic about the octant's centre
    const double *node_s;
};

// Host-side octree topology built from the block list.
struct Topology {
    int nbase = 0, vlev = 0, nblocks = 0, n_levels = 0, max_depth = 0, root = 0;
    double box = 0.0, box_lo[3] = {0.0, 0.0, 0.0};
    int64_t n_nodes = 0;
    std::vector<uint64_t> key;        // [n_nodes]
    std::vector<double> geom;         // [n_nodes][4]: centre x, y, z, edge
    std::vector<int32_t> child;       // [n_nodes]
    std::vector<int32_t> flags;       // [n_nodes] static FLAG_BOTTOM
    std::vector<int32_t> parent;      // [n_nodes], -1 for the root
    std::vector<LeafInfo> leaves;     // internal leaf order
    std::vector<int32_t> internal_of_canon;  // canonical leaf -> internal leaf
    std::vector<int32_t> combine_nodes;      // virtual + parent-block nodes (above the leaf blocks)
    // per combine node q: the range [first, end) of leaf ordinals below it
    std::vector<int32_t> combine_range;      // [combine_nodes.size()][2]
};

// Returns "" on success, else the reason the block list is rejected.
std::string build_topology(Topology &t, int n_blocks, const int32_t *level, const double *lo,
                           const int32_t *parent, const int32_t *child, const uint8_t *is_leaf,
                           const double box_lo[3], double box_size);

}  // namespace bh

struct bh_ctx {
    int device = -1;
    hipStream_t stream = nullptr;
    std::string err;
};

namespace bh {
constexpr int kBlockRow = 12;  // leaf-ordered copy of a block node's row: X Y Z M Q[6] S, pad
constexpr int kEwaldValues = 20;  // D, gradient (3), Hessian (6), third derivatives (10)
// The walks' table points, dimensionless: D L and gradient L^2, then Hessian
// L^3 and third derivatives L^4 at half the precision.  fp32 walks: 4 fp32 +
// 16 fp16 = 48 bytes (three 16-byte loads); fp64 walks: 4 fp64 + 16 fp32 =
// 96 bytes (six).
constexpr int kEwaldCompactFloats = 12;
constexpr int kEwaldCompactDoubles = 12;
constexpr int kEwaldNearTerms = 11;  // D0, the r^2 term, 9 terms of degree 4, 6 and 8
// default error budget of the group-centre cubic of D (per unit mass, units of 1/L; the table's own
// lookup bound is about 1.1e-6 at 33^3 points)
constexpr double kEwaldLocalBudget = BH_EWALD_LOCAL_BUDGET;
}

// Every handle records the device it was created on: its destroy call frees
// on that device without touching the context, which may already be gone.
struct bh_ewald {
    bh_ctx *ctx = nullptr;
    int device = -1;
    double L = 0.0;   // box side
    int n = 0;        // points per axis over [0, L/2]
    double sp = 0.0;  // spacing (L/2) / (n - 1)
    double *d_t64 = nullptr;   // [n^3][20] D and its derivatives to third order (export)
    // series of D L near the origin (|R| <= near_radius L), fitted at creation:
    // D0, 2 pi / 3, then the coefficients of e1^2, e2, e1^3, e1 e2, e3, e1^4,
    // e1^2 e2, e2^2, e1 e3 (e1 = X + Y + Z, e2 = XY + YZ + ZX, e3 = XYZ, X = (R_x / L)^2 ...)
    double near_coef[bh::kEwaldNearTerms] = {};
    double near_radius = 0.0;  // 0: not used (the fit missed its accuracy)
    double near_err = 0.0;     // largest |series - D L| at the check points
    float *d_near = nullptr;   // the coefficients in fp32, then near_radius^2
    double *d_t64c = nullptr;  // [n^3][12] compact rows of the fp64 walks and direct sum
    float *d_t32 = nullptr;    // [n^3][12] compact rows of the fp32 walks
    // worst-case error per unit mass (in units of 1/L) that the walks may add by summing D over a group
    // through one cubic about the group centre (0: every pair through its own table point)
    double local_budget = bh::kEwaldLocalBudget;
};

struct bh_grid {
    bh_ctx *ctx = nullptr;
    int device = -1;
    bh::Topology topo;
    int group_cells = bh::kGroupCells;
    int64_t n_groups = 0;
    int64_t n_units = 0;  // 64-cell octants, 8 per leaf block (dispatch units of the fused walks)
    int64_t n_cells = 0;
    // device copies of the static topology
    double *d_geom = nullptr;            // [n_nodes][4]
    int32_t *d_child = nullptr;          // [n_nodes]
    int32_t *d_flags = nullptr;          // [n_nodes]
    bh::LeafInfo *d_leaves = nullptr;    // [n_leaf]
    int32_t *d_internal_of_canon = nullptr;
    int32_t *d_combine = nullptr;
    int32_t *d_combine_range = nullptr;
    int32_t *d_parent = nullptr;         // [n_nodes]
    int32_t *d_leaf_parent = nullptr;    // [n_leaf] parent node of each leaf block's node (itself at the root)
};

struct bh_moments {
    const bh_grid *grid = nullptr;
    int device = -1;
    double *d_mom = nullptr;              // [n_nodes][kMom]
    double *d_s = nullptr;                // [n_nodes] sum m |r - X|^2
    double *d_brow = nullptr;             // [n_leaf][kBlockRow] each leaf block node's X Y Z M Q[6] S, leaf order
    bh::WalkRec32 *d_w32 = nullptr;
    bh::WalkRec64 *d_w64 = nullptr;
    bh::FarRec32 *d_f32 = nullptr;
    double4 *d_cell64 = nullptr;          // [n_cells] x, y, z, m (internal order)
    float4 *d_cell32 = nullptr;
    // d_flags[0]: epoch of the last moments build that saw an invalid density;
    // d_flags[1]: epoch of the last walk whose traversal stack overflowed.
    // Epoch stamps (atomicMax) replace clearing the flags before every call.
    int *d_flags = nullptr;
    int mom_epoch = 0;
    mutable int walk_epoch = 0;
    // dispatch schedule of the fused walks (single-grid calls): each fused
    // walk records the cost of every group; the next upward pass sorts the
    // groups by it into the order that the following fused walks dispatch
    float *d_theta = nullptr;     // [n_groups] canonical order: the learned step's thetas
    uint32_t *d_cost = nullptr;   // [n_units], internal octant order
    int32_t *d_order = nullptr;   // [n_units]
    int *d_sched = nullptr;       // bin histogram [256], placement cursors [256], finished count: zero between passes
    mutable bool cost_valid = false;  // d_cost holds a walk's costs
    bool order_valid = false;         // d_order holds a permutation
};

struct bh_lists {
    const bh_grid *grid = nullptr;
    int device = -1;
    int64_t cap_far = 0, cap_near = 0;
    int64_t n_far = 0, n_near = 0;
    int32_t *d_far = nullptr, *d_near = nullptr;         // node ids
    int64_t *d_far_off = nullptr, *d_near_off = nullptr;  // [n_groups + 1], internal group order
    int32_t *d_far_cnt = nullptr, *d_near_cnt = nullptr;  // [n_groups]
    int64_t *d_partials = nullptr;                        // scan block sums
    int64_t *d_status = nullptr;  // [4]: far total, near total, walk flag, density flag
    int64_t *h_status = nullptr;  // pinned copy of d_status
    int precision = BH_FP32;
};

namespace bh {
// kernel launchers (bh_kernels.hip); all enqueue on `s`.
// epoch > 0: stamp invalid densities with that value instead of a new epoch
// Upward pass.  schedule: also sort the groups by the costs that the last
// fused walk recorded, into the dispatch order of the next fused walks.
hipError_t launch_moments(const bh_grid *g, bh_moments *m, const double *rho, hipStream_t s, int epoch = 0,
                          bool schedule = false);
WalkArgs fused_args(const bh_grid *g, const bh_moments *m, double theta, const float *theta_group, int precision,
                    double G, double *phi, int32_t *counts, int epoch);
hipError_t launch_batch_reset(const WalkArgs *grids, int n, unsigned long long *counter, hipStream_t s);
// waves: kernel variant (fused_variant_exists), workgroups: persistent grid size
hipError_t launch_batch_walk_potential(const WalkArgs *grids, const int2 *order, int64_t total,
                                       unsigned long long *counter, int precision, int waves, int workgroups,
                                       hipStream_t s);
int fused_waves_per_simd(int precision);
bool fused_variant_exists(int precision, int waves);
// The periodic box's fields of a fused walk's arguments (table, near series, group-centre cubics, S).
void periodic_args(WalkArgs &a, const bh_grid *g, const bh_moments *m, const bh_ewald *e, int precision);
// Persistent periodic walk over a batch whose grids share one box; local: the cubic kernels.
int periodic_waves_per_simd(int precision, bool local);
hipError_t launch_batch_walk_potential_periodic(const WalkArgs *grids, const int2 *order, int64_t total,
                                                unsigned long long *counter, int precision, bool local,
                                                int workgroups, hipStream_t s);
hipError_t launch_walk(const bh_grid *g, const bh_moments *m, bh_lists *L, double theta, const float *theta_group,
                       int precision, bool fill, hipStream_t s);
hipError_t launch_scan(const bh_grid *g, const bh_moments *m, bh_lists *L, hipStream_t s);
// Periodic Green's function table, periodic fused walk + sums, periodic
// direct sum.
hipError_t launch_ewald_table(const bh_ewald *e, hipStream_t s);
hipError_t launch_ewald_points(double L, const double *u, int n, double *out, hipStream_t s);
hipError_t fit_ewald_near_series(bh_ewald *e, hipStream_t s);
// Largest cell side whose cubics of D stay within the table's budget:
// 32 (w + u)^4 <= budget (units of L), with w = sqrt(3) sp / (2L) the reach of
// a pair lookup and u = spread h / L the farthest cell centre from the
// cubic's centre: 1.5 sqrt(3) for the centre of a 4x4x4 octant, sqrt(3) / 2
// for the centre of a bottom node (2x2x2 cells).
constexpr double kLocalSpreadOctant = 1.5 * 1.7320508075688772, kLocalSpreadNode = 0.5 * 1.7320508075688772;
inline double ewald_local_hmax(const bh_ewald *e, double spread) {
    if (!(e->local_budget > 0.0)) return 0.0;
    const double reach = std::pow(e->local_budget / 32.0, 0.25);
    const double u = reach - std::sqrt(3.0) * 0.5 * e->sp / e->L;
    return u > 0.0 ? u * e->L / spread : 0.0;
}
hipError_t launch_walk_potential_periodic(const bh_grid *g, const bh_moments *m, const bh_ewald *e, double theta,
                                          const float *theta_group, int precision, double G, double *phi,
                                          int32_t *counts, hipStream_t s);
hipError_t launch_direct_periodic(const bh_grid *g, const bh_moments *m, const bh_ewald *e, const int64_t *targets,
                                  int64_t n, double G, double *out, hipStream_t s);
// The fused walk with a per-group theta array (a kernel of its own name).
hipError_t launch_walk_potential_theta(const bh_grid *g, const bh_moments *m, const float *theta_group,
                                       int precision, double G, double *phi, int32_t *counts, hipStream_t s);
hipError_t launch_walk_potential(const bh_grid *g, const bh_moments *m, double theta, const float *theta_group,
                                 int precision, double G, double *phi, int32_t *counts, hipStream_t s);
// fused walk with an opening test (BH_MAC_*) and far-field order (2 or 0)
hipError_t launch_walk_potential_opts(const bh_grid *g, const bh_moments *m, double theta, const float *theta_group,
                                      int precision, double G, double *phi, int32_t *counts, int mac, int order,
                                      hipStream_t s);
// walk fused with potential (phi may be NULL) and acceleration sums
hipError_t launch_walk_accel(const bh_grid *g, const bh_moments *m, double theta, const float *theta_group,
                             int precision, double G, double *phi, double *acc, int32_t *counts, hipStream_t s);
hipError_t launch_potential(const bh_grid *g, const bh_moments *m, const bh_lists *L, double G, int precision,
                            double *phi, hipStream_t s);
hipError_t launch_direct(const bh_grid *g, const bh_moments *m, const int64_t *targets, int64_t n, double G,
                         double *out, bool accel, hipStream_t s);
int walk_k8_threshold(int max_depth);
// Device address of the static scratch of bh_potential_static on `device`
// (looked up once per device; out may be NULL).
hipError_t static_scratch_setup(int device, void **out);
}  // namespace bh
