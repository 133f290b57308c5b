/*
 * bh.h -- C ABI of the MI355X (gfx950) Barnes-Hut gravitational potential
 * library for block-structured octree AMR meshes.
 *
 * The library computes, for every cell of an AMR mesh of 8^3-cell blocks, the
 * potential phi_i = -G sum_{j != i} m_j / |r_i - r_j| (Eq. 2 of the paper's
 * introduction, without its factor 1/2) approximated by the Barnes-Hut method
 * of section 2: an octree whose nodes carry mass, centre of mass and (beyond
 * the paper) a traceless quadrupole; a node is used as a whole when
 * d > l/theta + delta (Eq. THETA2) holds for every cell of a group of
 * neighbouring cells (the all() vote of the potential-kernel section).
 *
 * Calls in the order the method runs:
 *   bh_ctx_create -> bh_grid_create -> bh_build_moments -> bh_walk
 *   -> bh_potential  (bh_direct for the exact O(N^2) reference)
 *
 * Conventions for every entry point
 *  - Return value: BH_OK (0) or a negative BH_E* code; the message of the last
 *    failure on a context is returned by bh_last_error().  Nothing is thrown
 *    across the ABI.
 *  - Pointers named *_dev are device pointers on the context's GPU; every
 *    other pointer is host memory.  The caller owns all buffers it passes and
 *    the HIP stream; the library owns its opaque handles and their device
 *    workspaces, which bh_*_destroy releases.  Handles may be destroyed in
 *    any order, also after the context or grid they were made with (each
 *    frees on the device it was created on); no other call may use a handle
 *    whose context or grid is gone.
 *  - Work is enqueued on the context's stream and is asynchronous unless the
 *    description says that the call synchronises.
 *  - Cell-field layout ("caller layout"): fp64 [n_leaf][8][8][8] indexed
 *    [leaf][z][y][x] (x fastest), leaves numbered in the order they appear in
 *    the block list.  Canonical cell id = leaf*512 + z*64 + y*8 + x.
 *  - Group order ("canonical group order"): leaf-major, then the aligned
 *    Morton runs of group_cells cells inside the block (Morton bit 0 = x).
 *  - Results are deterministic for a fixed grid, input and parameter set.
 *  - Calls that use one moments handle must not overlap (issue them on one
 *    stream, or synchronise between streams): they share its device
 *    workspace (status flags, the per-group costs that each fused walk
 *    records, and the dispatch order built from them).
 */
#ifndef BH_H
#define BH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define BH_OK 0
#define BH_EINVAL (-1)     /* invalid argument or malformed grid */
#define BH_ENOMEM (-2)     /* host or device allocation failed */
#define BH_EDEVICE (-3)    /* a HIP runtime call failed (message has the hipError_t) */
#define BH_ECAPACITY (-4)  /* a fixed-size structure would overflow (message says which) */
#define BH_ESTATE (-5)     /* call out of order (e.g. moments of another grid) */

/* arithmetic of the walk and of the pair sums */
#define BH_FP64 0 /* everything in fp64 */
#define BH_FP32 1 /* fp32 opening tests and pair terms, fp64 accumulation per cell */

typedef struct bh_ctx bh_ctx;
typedef struct bh_grid bh_grid;
typedef struct bh_moments bh_moments;
typedef struct bh_lists bh_lists;
typedef struct bh_mlp bh_mlp;
typedef struct bh_batch bh_batch;
typedef struct bh_ewald bh_ewald;

/* ---------------------------------------------------------------- context */

/* Create a context on HIP device `device` that enqueues on `hip_stream`
 * (a hipStream_t; NULL = the null stream).  device = -1 creates a host-only
 * context: grids can be built and inspected (topology only), every GPU entry
 * point then fails with BH_ESTATE.  Errors: BH_EINVAL (bad device),
 * BH_EDEVICE, BH_ENOMEM. */
int bh_ctx_create(bh_ctx **ctx, int device, void *hip_stream);
/* Replace the stream used by later calls (the caller keeps ownership). */
int bh_ctx_set_stream(bh_ctx *ctx, void *hip_stream);
int bh_ctx_destroy(bh_ctx *ctx);
/* Message of the last failed call on ctx ("" if none).  Owned by ctx. */
const char *bh_last_error(const bh_ctx *ctx);
/* Message of the last failed bh_ctx_create in this process. */
const char *bh_create_error(void);

/* ---------------------------------------------------------------- grid (topology) */

/* Build the octree topology of an AMR mesh (section 3.1.1: cell data collected per
 * block, cells treated as point masses; tree nodes down to the cells as in
 * section 2).  Host arrays, all copied:
 *   level[n]      AMR level, 0 for the base blocks
 *   lo[n][3]      lower corner (fp64)
 *   parent[n]     parent block or -1 (base blocks)
 *   child[n][8]   children by octant o = ox + 2 oy + 4 oz, -1 for leaves
 *   is_leaf[n]    1 for leaf blocks (the ones carrying cells)
 * The base blocks must tile the box [box_lo, box_lo + box_size]^3 as an
 * nbase^3 lattice with nbase a power of two; log2(nbase) virtual levels join
 * them under one root.  nb must be 8 (cells per block edge).  group_cells is
 * the number of neighbouring cells sharing one opening vote and one
 * interaction list (the all() vote of section 3.3, whose group is a 32-thread
 * warp): 32, 64, 128, 256 or 512, an aligned Morton run of the block's cells
 * (4x4x2, 4x4x4, 8x4x4, 8x8x4 or the whole 8x8x8 block).  A group of 64 or
 * more cells spans group_cells/64 wavefronts that walk alike; two 32-cell
 * groups share one wavefront.  The learned-theta calls (features, network
 * inference, per-group errors) and batches need 64-cell groups.
 * Errors: BH_EINVAL with the first inconsistency found
 * (parent/child mismatch, level, position off the lattice, missing base block,
 * duplicate block, tree deeper than 18 levels), BH_ENOMEM, BH_EDEVICE. */
int bh_grid_create(bh_ctx *ctx, bh_grid **grid, int n_blocks, int nb, const int32_t *level, const double *lo,
                   const int32_t *parent, const int32_t *child, const uint8_t *is_leaf, const double box_lo[3],
                   double box_size, int group_cells);
int bh_grid_destroy(bh_grid *grid);

typedef struct {
    int64_t n_nodes;    /* octree nodes: virtual + blocks + in-block (octant, bottom) */
    int64_t n_leaf;     /* leaf blocks */
    int64_t n_cells;    /* 512 * n_leaf */
    int64_t n_groups;   /* n_cells / group_cells */
    int32_t group_cells;
    int32_t nbase;      /* base blocks per dimension */
    int32_t max_depth;  /* depth of the deepest bottom node (root = 0) */
    int32_t n_levels;   /* AMR levels present (max level + 1) */
} bh_grid_info_t;

int bh_grid_info(const bh_grid *grid, bh_grid_info_t *info);
/* Node identity shared with any other implementation: key = depth << 57 |
 * ix << 38 | iy << 19 | iz, with (ix, iy, iz) the node's lower corner in units
 * of its own edge box_size / 2^depth.  keys[n_nodes], indexed by node id. */
int bh_grid_node_keys(const bh_grid *grid, uint64_t *keys);

/* ---------------------------------------------------------------- moments */

/* Upward pass (section 3.2.3, the centers-of-gravitation kernel, extended to
 * quadrupoles): cell masses m = rho h^3 at the cell centres, then for every
 * node its mass M, centre of mass X = sum m r / M (Eq. R), traceless
 * quadrupole about X, Q = sum m (3 D D^T - |D|^2 I) (combined bottom-up with
 * the parallel-axis rule), and delta = |X - geometric centre| (Eq. THETA2).
 * Zero-mass nodes get X = centre, Q = 0, delta = 0 and are skipped by the walk.
 * rho_dev: fp64 caller layout, read only.  *m is created on first use (pass
 * *m == NULL) and reused when non-NULL (it must belong to `grid`).
 * Densities must be finite and >= 0: a violation is detected on the device;
 * bh_walk (or bh_moments_check) then fails with BH_EINVAL.
 * Dispatch schedule: once a fused walk (bh_walk_potential[_ex],
 * bh_walk_accel, bh_learned_walk_potential) has run on *m, this call also
 * sorts the groups by the work that walk recorded for each (heaviest first);
 * later fused walks start their groups in that order, which balances the
 * end of the launch and leaves every result unchanged bit for bit.  The sort
 * runs inside the moments kernels (no extra launch) and leaves no state that
 * a replay of a captured graph would have to reset. */
int bh_build_moments(bh_ctx *ctx, const bh_grid *grid, const double *rho_dev, bh_moments **m);
/* Synchronise and report device-side conditions: BH_EINVAL if the densities
 * seen by the last bh_build_moments were invalid, BH_ECAPACITY if the last walk
 * on these moments overflowed its traversal stack, else BH_OK. */
int bh_moments_check(bh_ctx *ctx, const bh_moments *m);
/* Synchronising host copy, by node id: M[n], X[n][3], Q[n][6] (xx yy zz xy xz
 * yz), delta[n].  Any pointer may be NULL. */
int bh_moments_export(bh_ctx *ctx, const bh_moments *m, double *M, double *X, double *Q, double *delta);
int bh_moments_destroy(bh_moments *m);

/* ---------------------------------------------------------------- walk */

/* Group tree walk (section 3.3, the potential kernel: depth-first traversal with
 * the all() vote over a group of neighbouring cells, Eq. THETA2 test
 * d^2 > (l/theta + delta)^2 at every cell of the group, equality opens).
 * Accepted nodes form the group's far list; rejected bottom nodes (2^3 cells)
 * its near list; other rejected nodes are opened.
 * theta: used for every group when theta_group_dev is NULL; must be in (0, 1].
 * theta_group_dev: NULL or fp32 [n_groups] in canonical group order, each in
 * (0, 1] (values outside are clamped into [1e-3, 1]).
 * precision: BH_FP64 or BH_FP32 arithmetic for the opening test.
 * *lists is created on first use and reused (grown as needed) when non-NULL.
 * Synchronises once (to size the lists).  Errors: BH_EINVAL (theta,
 * precision, or invalid densities seen by bh_build_moments), BH_ECAPACITY
 * (traversal stack), BH_ESTATE (m not built for grid), BH_ENOMEM, BH_EDEVICE. */
int bh_walk(bh_ctx *ctx, const bh_grid *grid, const bh_moments *m, double theta, const float *theta_group_dev,
            int precision, bh_lists **lists);
/* Totals of the last walk: far entries, near entries (bottom nodes). */
int bh_lists_info(const bh_lists *lists, int64_t *n_far, int64_t *n_near);
/* Synchronising host copy in canonical group order: far_off[n_groups + 1],
 * far_node[n_far], near_off[n_groups + 1], near_node[n_near] (node ids, see
 * bh_grid_node_keys).  Lists of one group keep the walk's order. */
int bh_lists_export(bh_ctx *ctx, const bh_lists *lists, int64_t *far_off, int32_t *far_node, int64_t *near_off,
                    int32_t *near_node);
int bh_lists_destroy(bh_lists *lists);

/* ---------------------------------------------------------------- sums */

/* Potential from the lists (section 3.3 accumulation, with quadrupoles):
 * phi_i = -G [ sum_far (M/d + R^T Q R / (2 d^5)) + sum_{near cells j != i} m_j / d ],
 * R = r_i - X.  precision BH_FP64: fp64 throughout; BH_FP32: fp32 pair terms
 * summed in fp32 over tiles of at most 64 nodes / 64 cells, tiles accumulated
 * in fp64.  phi_dev: fp64 caller layout, fully overwritten. */
int bh_potential(bh_ctx *ctx, const bh_grid *grid, const bh_moments *m, const bh_lists *lists, double G,
                 int precision, double *phi_dev);

/* Walk and potential in one pass (the same method and the same tiles, in the
 * same order, as bh_walk followed by bh_potential, hence the same bits), without
 * materialising the interaction lists and without synchronising: accepted
 * nodes and near bottom nodes are buffered per group in on-chip memory and
 * summed tile by tile as the traversal produces them.  Arguments as for
 * bh_walk / bh_potential.  counts_dev: NULL or int32 [n_groups][2] receiving
 * each group's far-node and near-bottom-node counts (canonical group order).
 * Device-side conditions (invalid densities, traversal stack overflow) are
 * reported by a later bh_moments_check. */
int bh_walk_potential(bh_ctx *ctx, const bh_grid *grid, const bh_moments *m, double theta,
                      const float *theta_group_dev, int precision, double G, double *phi_dev, int32_t *counts_dev);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc):
 * bh_build_moments followed by bh_walk_potential in one call that allocates
 * nothing.  The workspace a moments handle would own (node moments, walk and
 * far records, cell records, per-group costs) lives instead in one static
 * device array of BH_STATIC_SCRATCH_BYTES per GPU, held from the library's
 * load on that GPU until the process ends.  Same kernels and tiles as the
 * two-call path in the natural group order, hence the same potential bits.
 * rho_dev, theta, theta_group_dev, precision, G, phi_dev, counts_dev: as for
 * bh_build_moments and bh_walk_potential.
 * status_dev: NULL or int32 [2], cleared by the call, then status_dev[0] != 0
 * if some density was negative or not finite and status_dev[1] != 0 if the
 * traversal stack overflowed (NULL: these conditions are not reported).
 * Workspace of a grid: 232 B per node + 48 B per cell + 96 B per leaf block
 * + 4 B per group, each part rounded up to 256 B (about 82 B per cell; the
 * 1.4M-cell MacLaurin benchmark mesh needs about 115 MB).  A grid that needs
 * more fails with BH_ECAPACITY before any work is enqueued.
 * Every call on one GPU shares that GPU's array and leaves its contents
 * behind: calls that overlap on one GPU (several streams or threads without
 * ordering) race and give undefined results.  Errors: BH_EINVAL, BH_ESTATE
 * (grid of another device), BH_ECAPACITY, BH_EDEVICE. */
#define BH_STATIC_SCRATCH_BYTES (128u * 1024u * 1024u)
int bh_potential_static(bh_ctx *ctx, const bh_grid *grid, const double *rho_dev, double theta,
                        const float *theta_group_dev, int precision, double G, double *phi_dev, int32_t *counts_dev,
                        int32_t *status_dev);

/* Accelerations g = -grad phi from the same walk and tiles as
 * bh_walk_potential: the gradient of the far term (monopole and quadrupole)
 * and of the near pair terms, taken term by term (an extension of the method,
 * whose potential the paper computes; section 3.1 lists forces among what is
 * written back with it):
 *   far node:  g += G [ Q R / d^5 - (M / d^3 + (5/2) R^T Q R / d^7) R ]
 *   near cell: g -= G m_j (r_i - r_j) / |r_i - r_j|^3,   R = r_i - X.
 * acc_dev: fp64 [n_leaf][8][8][8][3] (x, y, z per cell, caller layout), fully
 * overwritten.  phi_dev: NULL, or receives the potential computed in the same
 * pass (the method's value; its rounding may differ from bh_walk_potential's
 * in the last fp32 bits, as the pair terms are evaluated in another order of
 * operations).  Other arguments, precisions, counts and errors as for
 * bh_walk_potential; tile sums in `precision`, accumulation in fp64. */
int bh_walk_accel(bh_ctx *ctx, const bh_grid *grid, const bh_moments *m, double theta, const float *theta_group_dev,
                  int precision, double G, double *phi_dev, double *acc_dev, int32_t *counts_dev);

/* The fused walk with the paper's own choices instead of this library's, for
 * comparison (both are beyond the default path, none changes the interface):
 *   mac   BH_MAC_CELLS (default): a node is accepted iff every cell of the
 *         group passes Eq. THETA2 (the all() vote of section 3.3, computed
 *         exactly in O(1) per node);
 *         BH_MAC_GROUP_BOX: iff the smallest distance d_c from the node's
 *         centre of mass to the group's cube (faces at the outer cell faces)
 *         passes it -- the test the paper uses between a node and a region
 *         (section 3.2, Fig. opening_angles2); stricter, so more work.
 *   order 2 (default): monopole + quadrupole far terms; 0: monopole only, the
 *         paper's far field.
 * Other arguments, outputs and errors as bh_walk_potential; opts NULL means
 * the defaults (then the result is bh_walk_potential's, bit for bit).
 * BH_EINVAL for an unknown mac or an order other than 0 or 2. */
#define BH_MAC_CELLS 0
#define BH_MAC_GROUP_BOX 1
typedef struct bh_walk_options {
    int32_t mac;
    int32_t order;
} bh_walk_options;

int bh_walk_potential_ex(bh_ctx *ctx, const bh_grid *grid, const bh_moments *m, double theta,
                         const float *theta_group_dev, int precision, double G, double *phi_dev, int32_t *counts_dev,
                         const bh_walk_options *opts);

/* Exact direct sum (Eq. 2) in fp64 at n_targets canonical cell ids
 * targets_dev[n] (int64, device); phi_dev[n] receives -G sum_{j != i} m_j/|r_ij|.
 * Uses the cell masses of the last bh_build_moments on m.  Errors: BH_EINVAL
 * (n_targets < 0), BH_ESTATE. */
int bh_direct(bh_ctx *ctx, const bh_grid *grid, const bh_moments *m, const int64_t *targets_dev,
              int64_t n_targets, double G, double *phi_dev);
/* Exact acceleration of the direct sum in fp64 at the same targets:
 * acc_dev[n][3] receives -G sum_{j != i} m_j (r_i - r_j) / |r_i - r_j|^3.
 * Arguments and errors as bh_direct. */
int bh_direct_accel(bh_ctx *ctx, const bh_grid *grid, const bh_moments *m, const int64_t *targets_dev,
                    int64_t n_targets, double G, double *acc_dev);

/* ---------------------------------------------------------------- periodic boxes
 *
 * Appendix "Periodic boundaries": in a box of side L repeated in every
 * direction, every contribution goes through the periodic Green's function
 * psi(r) = 1/|r| + D(r) (Ewald's split into short- and long-range sums, the
 * mean density removed).  This library tabulates the smooth part D on the
 * octant [0, L/2]^3 with its derivatives to third order and evaluates it by a
 * third-order Taylor expansion about the nearest table point (in place of the
 * paper's nested grids with quadratic interpolation of the whole field: the
 * singular 1/|r| is exact here, so one uniform grid suffices).
 *
 * The periodic walk and sum: every pair is taken at its nearest image, R
 * the nearest image of r_i - X.  A node is accepted iff the opening test of
 * bh_walk passes at every cell of the group with that distance; a far node
 * adds
 *   M (1/|R| + D(R)) + R^T Q R / (2 |R|^5) + Q:H(R) / 6 + 2 pi S / (3 L^3)
 * (H the Hessian of D, S = sum m |r - X|^2: the expansion of its cells'
 * periodic potentials to second order), a near cell m (1/|R| + D(R)),
 * the cell itself m D(0).  phi_i = -G (sum). */

/* Upper bound of n_points for bh_ewald_create. */
#define BH_EWALD_MAX_POINTS 129

/* Build the table for box side box_size on n_points^3 points (spacing
 * box_size / (2 (n_points - 1))) on the context's device and stream
 * (asynchronous).  It holds the fp64 values (160 bytes per point, what
 * bh_ewald_export returns) and the rows the walks read, dimensionless and
 * compact: D L and the gradient L^2 at the walk's precision, the Hessian L^3
 * and third derivatives L^4 at half of it (fp64 walks and the direct sum:
 * 96 bytes per point; fp32 walks: 48).  Errors:
 * BH_EINVAL (box_size <= 0 or not finite, n_points outside
 * [3, BH_EWALD_MAX_POINTS]), BH_ENOMEM, BH_EDEVICE. */
int bh_ewald_create(bh_ctx *ctx, double box_size, int n_points, bh_ewald **table);
int bh_ewald_destroy(bh_ewald *table);
/* Synchronising host copy of the fp64 table, values[n^3][20] indexed
 * ((k n + j) n + i) for the point (i, j, k) spacing: D; D_x D_y D_z;
 * D_xx D_yy D_zz D_xy D_xz D_yz; D_xxx D_yyy D_zzz D_xxy D_xxz D_xyy D_yyz
 * D_xzz D_yzz D_xyz. */
int bh_ewald_export(bh_ctx *ctx, const bh_ewald *table, double *values);
/* Number of values bh_ewald_near_series returns. */
#define BH_EWALD_NEAR_TERMS 11
/* The series of the smooth part D near the origin that the fp32 periodic
 * walks use for near-cell pairs within radius L of each other (appendix
 * "Periodic boundaries": D is smooth there, has the cube's symmetry and the
 * Laplacian 4 pi / L^3).  In units of L, with X = (R_x / L)^2, Y, Z and
 * e1 = X + Y + Z, e2 = XY + YZ + ZX, e3 = XYZ:
 *   D L = c0 + c1 e1 + c2 e1^2 + c3 e2 + c4 e1^3 + c5 e1 e2 + c6 e3
 *       + c7 e1^4 + c8 e1^2 e2 + c9 e2^2 + c10 e1 e3,
 * c0 = D(0) L and c1 = 2 pi / 3 from the Ewald sums, c2..c10 fitted to them by
 * least squares when the table is created.  coeffs[BH_EWALD_NEAR_TERMS]
 * (host): c0..c10; *radius (host): the radius in units of L within which the
 * walks use the series, 0 if the fit missed its accuracy and the table serves
 * every pair; *max_err (host): the largest |series - D L| found at the fit
 * points and a second set of check points.  Errors: BH_EINVAL (NULL). */
int bh_ewald_near_series(bh_ctx *ctx, const bh_ewald *table, double *coeffs, double *radius, double *max_err);
/* Error budget of the group-centre cubic in the periodic walks.  D is
 * smooth, so over the cells x = c + u near a centre c the sum over a group's
 * sources of m_s D(x - X_s) (and, for far nodes, the quadrupole's Hessian
 * term) is one cubic in u: each source's third-order expansion about its table
 * point (the same expansion a pair lookup makes) re-expanded about u = 0,
 * summed over the sources, and evaluated once per cell.  A pair then costs
 * what it costs without a box (1/|R| and the quadrupole).  The expansion
 * reaches |delta| <= sqrt(3) sp / 2 + |u|max instead of sqrt(3) sp / 2, so its
 * remainder grows; with |D^(4)| <= 24 / (L/2)^5 it is at most
 * 32 |delta / L|^4 / L per unit mass.  The centre is the wavefront's 4x4x4
 * octant's (|u| <= 1.5 sqrt(3) h; one table row per source) when that bound
 * stays within budget, else each bottom node's (2x2x2 cells, |u| <= sqrt(3)
 * h / 2; eight cubics per wavefront, one table row per source and bottom
 * node) when that one does, else every pair is looked up.  The budget is per
 * unit mass, in units of 1/L: at creation BH_EWALD_LOCAL_BUDGET, against about
 * 1.1e-6 for a 33^3 table's own lookup.  Only wavefronts holding one group
 * (group_cells >= 64) take a cubic, and a tile any of whose sources lies at
 * different nearest images from the octant's cells is summed pair by pair.
 * budget = 0: every pair through its own table point.  *h_max (host, may be
 * NULL): the largest cell side whose groups take a cubic, 0 for none.
 * Errors: BH_EINVAL (NULL table, budget negative or not finite). */
#define BH_EWALD_LOCAL_BUDGET 5e-5
int bh_ewald_set_local_budget(bh_ctx *ctx, bh_ewald *table, double budget, double *h_max);
/* Synchronising host copy of S = sum m |r - X|^2 of every node (by node id),
 * as built by the last bh_build_moments. */
int bh_moments_export_trace(bh_ctx *ctx, const bh_moments *m, double *S);
/* The periodic walk and sum (above) in one launch; arguments as
 * bh_walk_potential.  Groups of cells no larger than the table's budget
 * admits sum D through the group-centre cubic
 * (bh_ewald_set_local_budget).  The grid's box must be the table's (to 1e-12).  The
 * fused walks' dispatch order and cost records apply as for
 * bh_walk_potential.  Errors: BH_EINVAL (theta, precision, G, box size),
 * BH_ESTATE, BH_EDEVICE; stack overflow as bh_walk_potential. */
int bh_walk_potential_periodic(bh_ctx *ctx, const bh_grid *grid, const bh_moments *m, const bh_ewald *table,
                               double theta, const float *theta_group_dev, int precision, double G, double *phi_dev,
                               int32_t *counts_dev);
/* Periodic direct sum at canonical cell ids targets_dev[n] (fp64):
 * phi_dev[n] = -G [sum_{j != i} m_j / |R_ij| + sum_j m_j D(R_ij)], R_ij the
 * nearest image of r_i - r_j, D from the table.  Errors as bh_direct. */
int bh_direct_periodic(bh_ctx *ctx, const bh_grid *grid, const bh_moments *m, const bh_ewald *table,
                       const int64_t *targets_dev, int64_t n_targets, double G, double *phi_dev);

/* ---------------------------------------------------------------- batches
 *
 * Many independent grids solved together: the moments of every grid, then ONE
 * persistent launch of the fused walk + sums in which each wavefront takes the
 * next (grid, group) work item from an atomic queue until all are done.  The
 * method per group is exactly bh_walk_potential's (same tiles, same order, the
 * same bits).  A batch owns its own moments; all grids must belong to ctx and
 * have 64-cell groups (BH_EINVAL otherwise). */
#define BH_ORDER_NATURAL 0 /* grid by grid, groups in Morton order */
#define BH_ORDER_COST 1    /* most expensive groups first (counts of the last solve) */

int bh_batch_create(bh_ctx *ctx, bh_batch **batch, int n_grids, bh_grid *const *grids);
int bh_batch_destroy(bh_batch *batch);
int bh_batch_info(const bh_batch *batch, int *n_grids, int64_t *n_groups);
/* rho_dev[k] / phi_dev[k]: device pointers of grid k (caller layout); host arrays
 * of n_grids pointers.  theta_group_dev: NULL or a host array whose entries are
 * NULL (use theta) or device fp32 [n_groups_k].  Asynchronous; device-side
 * conditions are reported by bh_batch_check. */
int bh_batch_solve(bh_ctx *ctx, bh_batch *batch, const double *const *rho_dev, double *const *phi_dev, double theta,
                   const float *const *theta_group_dev, int precision, double G);
/* bh_batch_solve for grids that all lie in the periodic box of `table`
 * (bh_walk_potential_periodic's walk and sums, its group-centre cubics within
 * the table's budget), in one persistent launch.  Every grid's box must be the
 * table's (to 1e-12, BH_EINVAL otherwise).  The batch's own kernel variant and
 * launch settings for isolated solves do not apply; graphs are for isolated
 * solves only.  Results equal bh_walk_potential_periodic on each grid, bit for
 * bit.  Errors as bh_batch_solve; BH_EDEVICE (table on another device). */
int bh_batch_solve_periodic(bh_ctx *ctx, bh_batch *batch, const bh_ewald *table, const double *const *rho_dev,
                            double *const *phi_dev, double theta, const float *const *theta_group_dev, int precision,
                            double G);
/* Record the same solve as a graph (nothing runs yet); bh_batch_replay launches
 * it on the context's stream.  The graph keeps the buffers and parameters given
 * here; the moments' flags are cleared by a kernel inside the graph, not by a
 * memset, so replays are independent. */
int bh_batch_capture(bh_ctx *ctx, bh_batch *batch, const double *const *rho_dev, double *const *phi_dev,
                     double theta, const float *const *theta_group_dev, int precision, double G);
int bh_batch_replay(bh_ctx *ctx, bh_batch *batch);
/* Synchronise; BH_EINVAL (invalid density) or BH_ECAPACITY (stack) for the first
 * grid that reported one in the last solve or replay. */
int bh_batch_check(bh_ctx *ctx, const bh_batch *batch);
/* Synchronising host copy of the per-group far / near counts of the last solve:
 * counts[n_groups_total][2], grid by grid, canonical group order within a grid. */
int bh_batch_counts(bh_ctx *ctx, const bh_batch *batch, int32_t *counts);
/* Queue order for later solves (BH_ORDER_NATURAL or BH_ORDER_COST); drops a
 * captured graph. */
int bh_batch_schedule(bh_ctx *ctx, bh_batch *batch, int mode);
/* Persistent workgroups per compute unit (0 = the kernel's resident waves per
 * SIMD); a tuning knob, drops a captured graph. */
int bh_batch_set_launch(bh_ctx *ctx, bh_batch *batch, int workgroups_per_cu);

/* Launch configuration of a batch's persistent solve.  Order, width and
 * variant leave the results unchanged bit for bit (each group is still
 * computed by one wavefront with the same tiles in the same order); a stack
 * limit below the default changes the traversal order and so the order of
 * the far tiles: the same far and near sets, summed in another order.
 *   order             BH_ORDER_NATURAL or BH_ORDER_COST (cost uses the counts
 *                     of the last solve; before any solve it is the natural order)
 *   workgroups_per_cu persistent workgroups of 4 wavefronts per compute unit,
 *                     0 = one per resident slot of the kernel variant, <= 64
 *   waves_per_simd    kernel variant by register budget (the compiler fits the
 *                     kernel in 512 / waves VGPRs): fp32 4, 6 or 8; fp64 2 or 4;
 *                     0 = the precision's default (8 fp32, 4 fp64).  A value
 *                     with no variant for the solve's precision makes that
 *                     solve fail with BH_EINVAL.
 *   stack_limit       traversal stack policy: the walk pops whole sibling sets
 *                     (64 nodes a step) while its stack holds at most this many
 *                     entries and single sets beyond; 0 = the largest value that
 *                     cannot overflow for each grid's depth, else >= 8 and
 *                     clamped to that value.
 * bh_batch_configure drops a captured graph; BH_EINVAL for values out of range. */
typedef struct bh_batch_config {
    int32_t order;
    int32_t workgroups_per_cu;
    int32_t waves_per_simd;
    int32_t stack_limit;
} bh_batch_config;

int bh_batch_configure(bh_ctx *ctx, bh_batch *batch, const bh_batch_config *config);
int bh_batch_get_config(const bh_batch *batch, bh_batch_config *config);

/* Autotuner: solves the batch (arguments as bh_batch_solve) under every
 * candidate configuration -- each kernel variant of the precision x launch
 * widths {1, waves/2, waves} workgroups per CU x both queue orders x stack
 * limits {largest safe, 64} -- timing `reps` solves of each with HIP events
 * after one untimed solve, and applies the one with the smallest median time.
 * best (may be NULL) receives it and best_ms its median time.  table (may be
 * NULL) receives up to table_cap rows of every candidate tried and its median
 * time in ms; *n_table (may be NULL) the number of candidates.  Synchronises;
 * phi_dev holds the potentials of the last candidate's solve.
 * BH_EINVAL for reps < 1 or invalid solve arguments. */
typedef struct bh_batch_timing {
    bh_batch_config config;
    float ms;
} bh_batch_timing;

int bh_batch_autotune(bh_ctx *ctx, bh_batch *batch, const double *const *rho_dev, double *const *phi_dev,
                      double theta, const float *const *theta_group_dev, int precision, double G, int reps,
                      bh_batch_config *best, float *best_ms, bh_batch_timing *table, int table_cap, int *n_table);

/* ---------------------------------------------------------------- learned theta
 *
 * Beyond the paper (which uses one runtime theta): a small network predicts,
 * per group, the largest opening angle that keeps that group's RMS relative
 * potential error under a target; its output feeds theta_group_dev of
 * bh_walk / bh_walk_potential.
 *
 * Features (fp32 [n_groups][BH_MLP_INPUTS], canonical group order):
 *   0 log2(group cells); 1 log(M_group / M_root); 2 log(group edge / box);
 *   3 AMR level of the leaf block; 4 log(max / mean cell mass in the group);
 *   5, 6 log(delta/l + 1e-6) and log(|Q|_F / (M l^2) + 1e-6) of the group's own
 *   node; 7, 8 the same for its leaf block; 9, 10 for the block's parent node;
 *   11 log(mean group density / mean density of the leaf block).
 * Network: x' = (x - mean) * scale; h1 = tanh(W1 x' + b1) (64);
 *   h2 = tanh(W2 h1 + b2) (64); z = W3 . h2 + b3; theta = 0.2 + 0.8 sigmoid(z).
 * Parameter vector (fp32, BH_MLP_PARAMS): W1[64][12] | b1[64] | W2[64][64] |
 *   b2[64] | W3[64] | b3.  Initial values are supplied by the caller. */
#define BH_MLP_INPUTS 12
#define BH_MLP_HIDDEN 64
#define BH_MLP_PARAMS 5057

/* Group features from the moments of the last bh_build_moments on m.
 * feat_dev: fp32 [n_groups][12] (device), fully overwritten. */
int bh_group_features(bh_ctx *ctx, const bh_grid *grid, const bh_moments *m, float *feat_dev);
/* Per-group RMS of the relative error of phi against ref (both fp64 caller
 * layout, device): rms_dev[g] = sqrt(mean over the group's cells of
 * ((phi - ref) / ref)^2), fp32 [n_groups], canonical group order. */
int bh_group_rms_error(bh_ctx *ctx, const bh_grid *grid, const double *phi_dev, const double *ref_dev,
                       float *rms_dev);
/* Create a network from host parameters (BH_MLP_PARAMS floats, copied) and the
 * input normalisation mean[12], scale[12] (copied).  Adam state starts at 0. */
int bh_mlp_create(bh_ctx *ctx, bh_mlp **net, const float *params, const float *mean, const float *scale);
int bh_mlp_set_params(bh_ctx *ctx, bh_mlp *net, const float *params);
/* Smallest theta bh_theta_infer and bh_learned_walk_potential may return for
 * this network, snapped up to the grid 0.20, 0.25, ..., 1.00 (default 0.20,
 * the bottom of the grid).  A network trained on labels that never go below
 * some theta extrapolates badly under it, and the walk's cost grows steeply
 * as theta falls (the far-node count of a group goes roughly as 1/theta^3), so
 * a handful of groups pushed there by the output shift can cost more than the
 * rest of the grid; the floor is the smallest training label.  bh_mlp_forward
 * (the continuous, unsnapped output used in training) is not affected.
 * Returns BH_EINVAL unless 0.2 <= theta_floor <= 1.  Host-only; takes effect
 * for launches enqueued after the call. */
int bh_mlp_set_theta_floor(bh_ctx *ctx, bh_mlp *net, float theta_floor);
/* Synchronising host copy of the parameters. */
int bh_mlp_get_params(bh_ctx *ctx, const bh_mlp *net, float *params);
/* theta_dev[n] = clamp(network(feat_dev[n][12]) - theta_shift, 0.05, 1).
 * bf16 = 1: bf16 weights, inputs and hidden activations with fp32
 * accumulation; bf16 = 0: fp32.  theta_shift is a safety margin calibrated at
 * training time (0 gives the raw network output). */
int bh_mlp_forward(bh_ctx *ctx, const bh_mlp *net, const float *feat_dev, int64_t n, int bf16, float theta_shift,
                   float *theta_dev);
/* Per-group theta for a walk in one pass: the features of bh_group_features
 * fed to the bf16 network without storing them, the network's products on
 * the matrix cores (16 groups per wavefront).  The output equals
 * bh_mlp_forward with bf16 = 1 up to the fp32 rounding of the sums, and is
 * snapped up to the grid 0.20, 0.25, ..., 1.00 the labels are defined on.
 * theta_dev: fp32 [n_groups], canonical group order. */
int bh_theta_infer(bh_ctx *ctx, const bh_grid *grid, const bh_moments *m, const bh_mlp *net, float theta_shift,
                   float *theta_dev);
/* The whole learned-theta walk in one call: bh_theta_infer, then the walk
 * and sums of bh_walk_potential with those thetas (two launches on the
 * context's stream; the same bits as the two calls).  theta_dev: NULL (the
 * thetas go to a buffer of the moments handle), or fp32 [n_groups] receiving
 * the thetas used.  Other arguments and errors as bh_walk_potential. */
int bh_learned_walk_potential(bh_ctx *ctx, const bh_grid *grid, const bh_moments *m, const bh_mlp *net,
                              float theta_shift, int precision, double G, double *phi_dev, float *theta_dev,
                              int32_t *counts_dev);
/* Gradient of L = (1/n) sum (theta(x_s) - label_s)^2 with respect to the
 * parameters (fp32, deterministic order).  grad_dev: fp32 [BH_MLP_PARAMS];
 * loss_dev: NULL or fp32 [1] receiving L. */
int bh_mlp_grad(bh_ctx *ctx, bh_mlp *net, const float *feat_dev, const float *label_dev, int64_t n, float *grad_dev,
                float *loss_dev);
/* One Adam step (Kingma & Ba) on the parameters with gradient grad_dev. */
int bh_mlp_adam_step(bh_ctx *ctx, bh_mlp *net, const float *grad_dev, float lr, float beta1, float beta2, float eps);
int bh_mlp_destroy(bh_mlp *net);

#ifdef __cplusplus
}
#endif
#endif /* BH_H */
