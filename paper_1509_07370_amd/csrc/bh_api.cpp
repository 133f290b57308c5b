// C ABI of the Barnes-Hut library: argument checking, ownership of device
// workspaces, and the order of kernel launches.  Every step of the method
// runs in the HIP kernels of bh_kernels.hip; this file only marshals.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>

#include "bh_internal.h"

namespace {

thread_local std::string g_create_error;

int fail(bh_ctx *ctx, int code, const std::string &msg) {
    if (ctx) ctx->err = msg;
    return code;
}

int hip_fail(bh_ctx *ctx, hipError_t e, const char *what) {
    std::string msg = std::string(what) + ": " + hipGetErrorName(e) + " (" + hipGetErrorString(e) + ")";
    return fail(ctx, e == hipErrorOutOfMemory ? BH_ENOMEM : BH_EDEVICE, msg);
}

#define HIPX(ctx, expr, what)                          \
    do {                                               \
        hipError_t _e = (expr);                        \
        if (_e != hipSuccess) return hip_fail(ctx, _e, what); \
    } while (0)

template <typename T>
hipError_t dalloc(T **p, size_t count) {
    *p = nullptr;
    if (count == 0) count = 1;
    return hipMalloc((void **)p, count * sizeof(T));
}

int require_gpu(bh_ctx *ctx) {
    if (!ctx) return BH_EINVAL;
    if (ctx->device < 0) return fail(ctx, BH_ESTATE, "host-only context: no GPU work possible");
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return hip_fail(ctx, e, "hipSetDevice");
    return BH_OK;
}

void hfree(void *p) {
    if (p) (void)hipFree(p);
}

void free_grid_device(bh_grid *g) {
    hfree(g->d_geom);
    hfree(g->d_child);
    hfree(g->d_flags);
    hfree(g->d_leaves);
    hfree(g->d_internal_of_canon);
    hfree(g->d_combine);
    hfree(g->d_combine_range);
    hfree(g->d_parent);
    hfree(g->d_leaf_parent);
    g->d_parent = nullptr;
    g->d_leaf_parent = nullptr;
    g->d_geom = nullptr;
    g->d_child = g->d_flags = g->d_internal_of_canon = g->d_combine = nullptr;
    g->d_combine_range = nullptr;
    g->d_leaves = nullptr;
}

}  // namespace

extern "C" {

const char *bh_create_error(void) { return g_create_error.c_str(); }

int bh_ctx_create(bh_ctx **out, int device, void *stream) {
    if (!out) return BH_EINVAL;
    *out = nullptr;
    if (device >= 0) {
        int n = 0;
        hipError_t e = hipGetDeviceCount(&n);
        if (e != hipSuccess) {
            g_create_error = std::string("hipGetDeviceCount: ") + hipGetErrorString(e);
            return BH_EDEVICE;
        }
        if (device >= n) {
            g_create_error = "device index out of range";
            return BH_EINVAL;
        }
        e = hipSetDevice(device);
        if (e != hipSuccess) {
            g_create_error = std::string("hipSetDevice: ") + hipGetErrorString(e);
            return BH_EDEVICE;
        }
        // the static scratch of bh_potential_static: its device address, once per device
        e = bh::static_scratch_setup(device, nullptr);
        if (e != hipSuccess) {
            g_create_error = std::string("static scratch address: ") + hipGetErrorString(e);
            return BH_EDEVICE;
        }
    } else if (device != -1) {
        g_create_error = "device must be >= 0, or -1 for a host-only context";
        return BH_EINVAL;
    }
    bh_ctx *c = new (std::nothrow) bh_ctx();
    if (!c) return BH_ENOMEM;
    c->device = device;
    c->stream = (hipStream_t)stream;
    *out = c;
    return BH_OK;
}

int bh_ctx_set_stream(bh_ctx *ctx, void *stream) {
    if (!ctx) return BH_EINVAL;
    ctx->stream = (hipStream_t)stream;
    return BH_OK;
}

int bh_ctx_destroy(bh_ctx *ctx) {
    delete ctx;
    return BH_OK;
}

const char *bh_last_error(const bh_ctx *ctx) { return ctx ? ctx->err.c_str() : "null context"; }

// ------------------------------------------------------------------ grid

int bh_grid_create(bh_ctx *ctx, bh_grid **out, int n_blocks, int nb, const int32_t *level, const double *lo,
                   const int32_t *parent, const int32_t *child, const uint8_t *is_leaf, const double box_lo[3],
                   double box_size, int group_cells) {
    if (!ctx) return BH_EINVAL;
    if (!out) return fail(ctx, BH_EINVAL, "grid output pointer is NULL");
    *out = nullptr;
    if (nb != bh::kNB) return fail(ctx, BH_EINVAL, "nb must be 8 (cells per block edge)");
    if (group_cells != 32 && group_cells != 64 && group_cells != 128 && group_cells != 256 && group_cells != 512)
        return fail(ctx, BH_EINVAL, "group_cells must be 32, 64, 128, 256 or 512");
    if (!level || !lo || !parent || !child || !is_leaf || !box_lo)
        return fail(ctx, BH_EINVAL, "a grid array pointer is NULL");
    bh_grid *g = new (std::nothrow) bh_grid();
    if (!g) return fail(ctx, BH_ENOMEM, "host allocation of the grid");
    g->ctx = ctx;
    g->device = ctx->device;
    std::string why;
    try {
        why = bh::build_topology(g->topo, n_blocks, level, lo, parent, child, is_leaf, box_lo, box_size);
    } catch (const std::bad_alloc &) {
        delete g;
        return fail(ctx, BH_ENOMEM, "host allocation while building the topology");
    }
    if (!why.empty()) {
        delete g;
        return fail(ctx, BH_EINVAL, "invalid grid: " + why);
    }
    if (bh::walk_k8_threshold(g->topo.max_depth) < 1) {
        delete g;
        return fail(ctx, BH_ECAPACITY, "tree too deep for the walk stack");
    }
    g->group_cells = group_cells;
    g->n_cells = (int64_t)g->topo.leaves.size() * bh::kCellsPerBlock;
    g->n_groups = g->n_cells / group_cells;
    g->n_units = (int64_t)g->topo.leaves.size() * 8;
    if (ctx->device >= 0) {
        int rc = require_gpu(ctx);
        if (rc) {
            delete g;
            return rc;
        }
        const auto &t = g->topo;
        std::vector<int32_t> leaf_parent(t.leaves.size());
        for (size_t f = 0; f < t.leaves.size(); f++) {
            const int b = t.leaves[f].block_node, p = t.parent[b];
            leaf_parent[f] = p >= 0 ? p : b;
        }
        hipError_t e;
        if ((e = dalloc(&g->d_geom, t.geom.size())) != hipSuccess ||
            (e = dalloc(&g->d_child, t.child.size())) != hipSuccess ||
            (e = dalloc(&g->d_flags, t.flags.size())) != hipSuccess ||
            (e = dalloc(&g->d_leaves, t.leaves.size())) != hipSuccess ||
            (e = dalloc(&g->d_internal_of_canon, t.internal_of_canon.size())) != hipSuccess ||
            (e = dalloc(&g->d_combine, t.combine_nodes.size())) != hipSuccess ||
            (e = dalloc(&g->d_combine_range, t.combine_range.size())) != hipSuccess ||
            (e = dalloc(&g->d_parent, t.parent.size())) != hipSuccess ||
            (e = dalloc(&g->d_leaf_parent, leaf_parent.size())) != hipSuccess) {
            free_grid_device(g);
            delete g;
            return hip_fail(ctx, e, "device allocation of the grid topology");
        }
        struct {
            void *d;
            const void *h;
            size_t n;
        } up[] = {{g->d_geom, t.geom.data(), t.geom.size() * sizeof(double)},
                  {g->d_child, t.child.data(), t.child.size() * sizeof(int32_t)},
                  {g->d_flags, t.flags.data(), t.flags.size() * sizeof(int32_t)},
                  {g->d_leaves, t.leaves.data(), t.leaves.size() * sizeof(bh::LeafInfo)},
                  {g->d_internal_of_canon, t.internal_of_canon.data(), t.internal_of_canon.size() * sizeof(int32_t)},
                  {g->d_combine, t.combine_nodes.data(), t.combine_nodes.size() * sizeof(int32_t)},
                  {g->d_combine_range, t.combine_range.data(), t.combine_range.size() * sizeof(int32_t)},
                  {g->d_parent, t.parent.data(), t.parent.size() * sizeof(int32_t)},
                  {g->d_leaf_parent, leaf_parent.data(), leaf_parent.size() * sizeof(int32_t)}};
        for (auto &u : up) {
            if (u.n == 0) continue;
            e = hipMemcpy(u.d, u.h, u.n, hipMemcpyHostToDevice);
            if (e != hipSuccess) {
                free_grid_device(g);
                delete g;
                return hip_fail(ctx, e, "upload of the grid topology");
            }
        }
    }
    *out = g;
    return BH_OK;
}

int bh_grid_destroy(bh_grid *g) {
    if (!g) return BH_OK;
    if (g->device >= 0) {
        (void)hipSetDevice(g->device);
        free_grid_device(g);
    }
    delete g;
    return BH_OK;
}

int bh_grid_info(const bh_grid *g, bh_grid_info_t *info) {
    if (!g || !info) return BH_EINVAL;
    info->n_nodes = g->topo.n_nodes;
    info->n_leaf = (int64_t)g->topo.leaves.size();
    info->n_cells = g->n_cells;
    info->n_groups = g->n_groups;
    info->group_cells = g->group_cells;
    info->nbase = g->topo.nbase;
    info->max_depth = g->topo.max_depth;
    info->n_levels = g->topo.n_levels;
    return BH_OK;
}

int bh_grid_node_keys(const bh_grid *g, uint64_t *keys) {
    if (!g || !keys) return BH_EINVAL;
    std::memcpy(keys, g->topo.key.data(), g->topo.key.size() * sizeof(uint64_t));
    return BH_OK;
}

// ------------------------------------------------------------------ moments

int bh_moments_destroy(bh_moments *m) {
    if (!m) return BH_OK;
    if (m->device >= 0) (void)hipSetDevice(m->device);
    hfree(m->d_mom);
    hfree(m->d_s);
    hfree(m->d_brow);
    hfree(m->d_w32);
    hfree(m->d_w64);
    hfree(m->d_f32);
    hfree(m->d_cell64);
    hfree(m->d_cell32);
    hfree(m->d_flags);
    hfree(m->d_cost);
    hfree(m->d_order);
    hfree(m->d_theta);
    hfree(m->d_sched);
    delete m;
    return BH_OK;
}

int bh_build_moments(bh_ctx *ctx, const bh_grid *g, const double *rho, bh_moments **mp) {
    int rc = require_gpu(ctx);
    if (rc) return rc;
    if (!g || !mp) return fail(ctx, BH_EINVAL, "grid or moments pointer is NULL");
    if (!rho) return fail(ctx, BH_EINVAL, "rho_dev is NULL");
    bh_moments *m = *mp;
    if (m && m->grid != g) return fail(ctx, BH_ESTATE, "moments handle belongs to another grid");
    if (!m) {
        m = new (std::nothrow) bh_moments();
        if (!m) return fail(ctx, BH_ENOMEM, "host allocation of the moments handle");
        m->grid = g;
        m->device = g->device;
        const int64_t nn = g->topo.n_nodes, nc = g->n_cells;
        hipError_t e;
        if ((e = dalloc(&m->d_mom, (size_t)nn * bh::kMom)) != hipSuccess || (e = dalloc(&m->d_s, (size_t)nn)) != hipSuccess ||
            (e = dalloc(&m->d_brow, g->topo.leaves.size() * bh::kBlockRow)) != hipSuccess ||
            (e = dalloc(&m->d_w32, (size_t)nn)) != hipSuccess || (e = dalloc(&m->d_w64, (size_t)nn)) != hipSuccess ||
            (e = dalloc(&m->d_f32, (size_t)nn)) != hipSuccess || (e = dalloc(&m->d_cell64, (size_t)nc)) != hipSuccess ||
            (e = dalloc(&m->d_cell32, (size_t)nc)) != hipSuccess || (e = dalloc(&m->d_flags, 2)) != hipSuccess ||
            (e = hipMemset(m->d_flags, 0, 2 * sizeof(int))) != hipSuccess ||
            (e = dalloc(&m->d_cost, (size_t)g->n_units)) != hipSuccess ||
            (e = dalloc(&m->d_theta, (size_t)g->n_groups)) != hipSuccess ||
            (e = dalloc(&m->d_order, (size_t)g->n_units)) != hipSuccess ||
            (e = dalloc(&m->d_sched, 2 * 256 + 1)) != hipSuccess ||
            (e = hipMemset(m->d_sched, 0, (2 * 256 + 1) * sizeof(int))) != hipSuccess) {
            bh_moments_destroy(m);
            return hip_fail(ctx, e, "device allocation of the moments");
        }
        *mp = m;
    }
    // once a fused walk has recorded its costs, the upward pass also sorts the
    // groups by them, for the dispatch order of the next fused walks
    const bool schedule = m->cost_valid && g->n_units > 1;
    HIPX(ctx, bh::launch_moments(g, m, rho, ctx->stream, 0, schedule), "moments kernels");
    if (schedule) m->order_valid = true;
    return BH_OK;
}

int bh_moments_check(bh_ctx *ctx, const bh_moments *m) {
    int rc = require_gpu(ctx);
    if (rc) return rc;
    if (!m) return fail(ctx, BH_EINVAL, "moments handle is NULL");
    int flags[2] = {0, 0};
    HIPX(ctx, hipMemcpyAsync(flags, m->d_flags, sizeof(flags), hipMemcpyDeviceToHost, ctx->stream), "copy flags");
    HIPX(ctx, hipStreamSynchronize(ctx->stream), "synchronise");
    if (m->mom_epoch > 0 && flags[0] == m->mom_epoch) return fail(ctx, BH_EINVAL, "densities must be finite and >= 0");
    if (m->walk_epoch > 0 && flags[1] == m->walk_epoch) return fail(ctx, BH_ECAPACITY, "walk stack overflow");
    return BH_OK;
}

int bh_moments_export(bh_ctx *ctx, const bh_moments *m, double *M, double *X, double *Q, double *delta) {
    int rc = require_gpu(ctx);
    if (rc) return rc;
    if (!m) return fail(ctx, BH_EINVAL, "moments handle is NULL");
    const int64_t nn = m->grid->topo.n_nodes;
    double *h = new (std::nothrow) double[(size_t)nn * bh::kMom];
    if (!h) return fail(ctx, BH_ENOMEM, "host buffer for the export");
    hipError_t e = hipMemcpyAsync(h, m->d_mom, (size_t)nn * bh::kMom * sizeof(double), hipMemcpyDeviceToHost,
                                  ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) {
        delete[] h;
        return hip_fail(ctx, e, "copy of the moments");
    }
    for (int64_t n = 0; n < nn; n++) {
        const double *r = h + n * bh::kMom;
        if (M) M[n] = r[3];
        if (X)
            for (int d = 0; d < 3; d++) X[3 * n + d] = r[d];
        if (Q)
            for (int c = 0; c < 6; c++) Q[6 * n + c] = r[4 + c];
        if (delta) delta[n] = r[10];
    }
    delete[] h;
    return BH_OK;
}

// ------------------------------------------------------------------ walk

int bh_lists_destroy(bh_lists *L) {
    if (!L) return BH_OK;
    if (L->device >= 0) (void)hipSetDevice(L->device);
    hfree(L->d_far);
    hfree(L->d_near);
    hfree(L->d_far_off);
    hfree(L->d_near_off);
    hfree(L->d_far_cnt);
    hfree(L->d_near_cnt);
    hfree(L->d_partials);
    hfree(L->d_status);
    if (L->h_status) (void)hipHostFree(L->h_status);
    delete L;
    return BH_OK;
}

int bh_walk(bh_ctx *ctx, const bh_grid *g, const bh_moments *m, double theta, const float *theta_group,
            int precision, bh_lists **lp) {
    int rc = require_gpu(ctx);
    if (rc) return rc;
    if (!g || !m || !lp) return fail(ctx, BH_EINVAL, "grid, moments or lists pointer is NULL");
    if (m->grid != g) return fail(ctx, BH_ESTATE, "moments were built for another grid");
    if (precision != BH_FP64 && precision != BH_FP32) return fail(ctx, BH_EINVAL, "precision must be BH_FP64 or BH_FP32");
    if (!theta_group && !(theta > 0.0 && theta <= 1.0)) return fail(ctx, BH_EINVAL, "theta must be in (0, 1]");
    bh_lists *L = *lp;
    if (L && L->grid != g) return fail(ctx, BH_ESTATE, "lists handle belongs to another grid");
    const int64_t ng = g->n_groups;
    if (!L) {
        L = new (std::nothrow) bh_lists();
        if (!L) return fail(ctx, BH_ENOMEM, "host allocation of the lists handle");
        L->grid = g;
        L->device = g->device;
        const int nblocks = (int)((ng + 1023) / 1024);
        hipError_t e;
        if ((e = dalloc(&L->d_far_off, (size_t)ng + 1)) != hipSuccess ||
            (e = dalloc(&L->d_near_off, (size_t)ng + 1)) != hipSuccess ||
            (e = dalloc(&L->d_far_cnt, (size_t)ng)) != hipSuccess ||
            (e = dalloc(&L->d_near_cnt, (size_t)ng)) != hipSuccess ||
            (e = dalloc(&L->d_partials, (size_t)2 * nblocks)) != hipSuccess ||
            (e = dalloc(&L->d_status, 4)) != hipSuccess ||
            (e = hipHostMalloc((void **)&L->h_status, 4 * sizeof(int64_t), hipHostMallocDefault)) != hipSuccess) {
            bh_lists_destroy(L);
            return hip_fail(ctx, e, "allocation of the list offsets");
        }
        *lp = L;
    }
    L->precision = precision;
    hipStream_t s = ctx->stream;
    m->walk_epoch++;
    HIPX(ctx, bh::launch_walk(g, m, L, theta, theta_group, precision, false, s), "walk (count pass)");
    HIPX(ctx, bh::launch_scan(g, m, L, s), "list offsets");
    HIPX(ctx, hipMemcpyAsync(L->h_status, L->d_status, 4 * sizeof(int64_t), hipMemcpyDeviceToHost, s), "status");
    HIPX(ctx, hipStreamSynchronize(s), "synchronise after the count pass");
    if (m->mom_epoch > 0 && L->h_status[3] == m->mom_epoch)
        return fail(ctx, BH_EINVAL, "densities must be finite and >= 0");
    if (L->h_status[2] == m->walk_epoch) return fail(ctx, BH_ECAPACITY, "walk stack overflow");
    const int64_t nf = L->h_status[0], nn = L->h_status[1];
    if (nf > L->cap_far) {
        hfree(L->d_far);
        L->d_far = nullptr;
        L->cap_far = 0;
        int64_t cap = nf + nf / 8 + 64;
        HIPX(ctx, dalloc(&L->d_far, (size_t)cap), "allocation of the far lists");
        L->cap_far = cap;
    }
    if (nn > L->cap_near) {
        hfree(L->d_near);
        L->d_near = nullptr;
        L->cap_near = 0;
        int64_t cap = nn + nn / 8 + 64;
        HIPX(ctx, dalloc(&L->d_near, (size_t)cap), "allocation of the near lists");
        L->cap_near = cap;
    }
    L->n_far = nf;
    L->n_near = nn;
    HIPX(ctx, bh::launch_walk(g, m, L, theta, theta_group, precision, true, s), "walk (fill pass)");
    return BH_OK;
}

int bh_lists_info(const bh_lists *L, int64_t *n_far, int64_t *n_near) {
    if (!L) return BH_EINVAL;
    if (n_far) *n_far = L->n_far;
    if (n_near) *n_near = L->n_near;
    return BH_OK;
}

int bh_lists_export(bh_ctx *ctx, const bh_lists *L, int64_t *far_off, int32_t *far_node, int64_t *near_off,
                    int32_t *near_node) {
    int rc = require_gpu(ctx);
    if (rc) return rc;
    if (!L || !far_off || !near_off) return fail(ctx, BH_EINVAL, "lists handle or offset buffer is NULL");
    const bh_grid *g = L->grid;
    const int64_t ng = g->n_groups;
    std::vector<int64_t> fo(ng + 1), no(ng + 1);
    std::vector<int32_t> fa(L->n_far > 0 ? L->n_far : 1), na(L->n_near > 0 ? L->n_near : 1);
    hipStream_t s = ctx->stream;
    HIPX(ctx, hipMemcpyAsync(fo.data(), L->d_far_off, (ng + 1) * sizeof(int64_t), hipMemcpyDeviceToHost, s), "copy");
    HIPX(ctx, hipMemcpyAsync(no.data(), L->d_near_off, (ng + 1) * sizeof(int64_t), hipMemcpyDeviceToHost, s), "copy");
    if (L->n_far)
        HIPX(ctx, hipMemcpyAsync(fa.data(), L->d_far, L->n_far * sizeof(int32_t), hipMemcpyDeviceToHost, s), "copy");
    if (L->n_near)
        HIPX(ctx, hipMemcpyAsync(na.data(), L->d_near, L->n_near * sizeof(int32_t), hipMemcpyDeviceToHost, s), "copy");
    HIPX(ctx, hipStreamSynchronize(s), "synchronise");
    // internal group g = f*8 + sub -> canonical group canon(f)*8 + sub
    const auto &leaves = g->topo.leaves;
    const int per = bh::kCellsPerBlock / g->group_cells;
    std::vector<int64_t> cf(ng), cn(ng);
    for (int64_t q = 0; q < ng; q++) {
        int64_t c = (int64_t)leaves[q / per].canon * per + q % per;
        cf[c] = fo[q + 1] - fo[q];
        cn[c] = no[q + 1] - no[q];
    }
    far_off[0] = near_off[0] = 0;
    for (int64_t c = 0; c < ng; c++) {
        far_off[c + 1] = far_off[c] + cf[c];
        near_off[c + 1] = near_off[c] + cn[c];
    }
    for (int64_t q = 0; q < ng; q++) {
        int64_t c = (int64_t)leaves[q / per].canon * per + q % per;
        if (far_node)
            std::memcpy(far_node + far_off[c], fa.data() + fo[q], (size_t)(fo[q + 1] - fo[q]) * sizeof(int32_t));
        if (near_node)
            std::memcpy(near_node + near_off[c], na.data() + no[q], (size_t)(no[q + 1] - no[q]) * sizeof(int32_t));
    }
    return BH_OK;
}

// ------------------------------------------------------------------ sums

int bh_potential(bh_ctx *ctx, const bh_grid *g, const bh_moments *m, const bh_lists *L, double G, int precision,
                 double *phi) {
    int rc = require_gpu(ctx);
    if (rc) return rc;
    if (!g || !m || !L || !phi) return fail(ctx, BH_EINVAL, "grid, moments, lists or phi_dev is NULL");
    if (m->grid != g || L->grid != g) return fail(ctx, BH_ESTATE, "moments or lists belong to another grid");
    if (precision != BH_FP64 && precision != BH_FP32) return fail(ctx, BH_EINVAL, "precision must be BH_FP64 or BH_FP32");
    if (!std::isfinite(G)) return fail(ctx, BH_EINVAL, "G must be finite");
    HIPX(ctx, bh::launch_potential(g, m, L, G, precision, phi, ctx->stream), "potential kernel");
    return BH_OK;
}

int bh_walk_potential(bh_ctx *ctx, const bh_grid *g, const bh_moments *m, double theta, const float *theta_group,
                      int precision, double G, double *phi, int32_t *counts) {
    int rc = require_gpu(ctx);
    if (rc) return rc;
    if (!g || !m || !phi) return fail(ctx, BH_EINVAL, "grid, moments or phi_dev is NULL");
    if (m->grid != g) return fail(ctx, BH_ESTATE, "moments were built for another grid");
    if (precision != BH_FP64 && precision != BH_FP32) return fail(ctx, BH_EINVAL, "precision must be BH_FP64 or BH_FP32");
    if (!theta_group && !(theta > 0.0 && theta <= 1.0)) return fail(ctx, BH_EINVAL, "theta must be in (0, 1]");
    if (!std::isfinite(G)) return fail(ctx, BH_EINVAL, "G must be finite");
    m->walk_epoch++;
    HIPX(ctx, bh::launch_walk_potential(g, m, theta, theta_group, precision, G, phi, counts, ctx->stream),
         "fused walk + potential kernel");
    return BH_OK;
}

int bh_walk_potential_ex(bh_ctx *ctx, const bh_grid *g, const bh_moments *m, double theta, const float *theta_group,
                         int precision, double G, double *phi, int32_t *counts, const bh_walk_options *opts) {
    int rc = require_gpu(ctx);
    if (rc) return rc;
    if (!g || !m || !phi) return fail(ctx, BH_EINVAL, "grid, moments or phi_dev is NULL");
    if (m->grid != g) return fail(ctx, BH_ESTATE, "moments were built for another grid");
    if (precision != BH_FP64 && precision != BH_FP32) return fail(ctx, BH_EINVAL, "precision must be BH_FP64 or BH_FP32");
    if (!theta_group && !(theta > 0.0 && theta <= 1.0)) return fail(ctx, BH_EINVAL, "theta must be in (0, 1]");
    if (!std::isfinite(G)) return fail(ctx, BH_EINVAL, "G must be finite");
    const int mac = opts ? opts->mac : BH_MAC_CELLS, order = opts ? opts->order : 2;
    if (mac != BH_MAC_CELLS && mac != BH_MAC_GROUP_BOX) return fail(ctx, BH_EINVAL, "unknown opening test (mac)");
    if (order != 0 && order != 2) return fail(ctx, BH_EINVAL, "order must be 0 or 2");
    m->walk_epoch++;
    HIPX(ctx, bh::launch_walk_potential_opts(g, m, theta, theta_group, precision, G, phi, counts, mac, order,
                                             ctx->stream),
         "fused walk + potential kernel");
    return BH_OK;
}

int bh_walk_accel(bh_ctx *ctx, const bh_grid *g, const bh_moments *m, double theta, const float *theta_group,
                  int precision, double G, double *phi, double *acc, int32_t *counts) {
    int rc = require_gpu(ctx);
    if (rc) return rc;
    if (!g || !m || !acc) return fail(ctx, BH_EINVAL, "grid, moments or acc_dev is NULL");
    if (m->grid != g) return fail(ctx, BH_ESTATE, "moments were built for another grid");
    if (precision != BH_FP64 && precision != BH_FP32) return fail(ctx, BH_EINVAL, "precision must be BH_FP64 or BH_FP32");
    if (!theta_group && !(theta > 0.0 && theta <= 1.0)) return fail(ctx, BH_EINVAL, "theta must be in (0, 1]");
    if (!std::isfinite(G)) return fail(ctx, BH_EINVAL, "G must be finite");
    m->walk_epoch++;
    HIPX(ctx, bh::launch_walk_accel(g, m, theta, theta_group, precision, G, phi, acc, counts, ctx->stream),
         "fused walk + acceleration kernel");
    return BH_OK;
}

int bh_direct(bh_ctx *ctx, const bh_grid *g, const bh_moments *m, const int64_t *targets, int64_t n, double G,
              double *phi) {
    int rc = require_gpu(ctx);
    if (rc) return rc;
    if (!g || !m) return fail(ctx, BH_EINVAL, "grid or moments is NULL");
    if (m->grid != g) return fail(ctx, BH_ESTATE, "moments belong to another grid");
    if (n < 0) return fail(ctx, BH_EINVAL, "n_targets must be >= 0");
    if (n > 0 && (!targets || !phi)) return fail(ctx, BH_EINVAL, "targets_dev or phi_dev is NULL");
    if (!std::isfinite(G)) return fail(ctx, BH_EINVAL, "G must be finite");
    HIPX(ctx, bh::launch_direct(g, m, targets, n, G, phi, false, ctx->stream), "direct-sum kernel");
    return BH_OK;
}

int bh_direct_accel(bh_ctx *ctx, const bh_grid *g, const bh_moments *m, const int64_t *targets, int64_t n, double G,
                    double *acc) {
    int rc = require_gpu(ctx);
    if (rc) return rc;
    if (!g || !m) return fail(ctx, BH_EINVAL, "grid or moments is NULL");
    if (m->grid != g) return fail(ctx, BH_ESTATE, "moments belong to another grid");
    if (n < 0) return fail(ctx, BH_EINVAL, "n_targets must be >= 0");
    if (n > 0 && (!targets || !acc)) return fail(ctx, BH_EINVAL, "targets_dev or acc_dev is NULL");
    if (!std::isfinite(G)) return fail(ctx, BH_EINVAL, "G must be finite");
    HIPX(ctx, bh::launch_direct(g, m, targets, n, G, acc, true, ctx->stream), "direct-sum acceleration kernel");
    return BH_OK;
}

// ------------------------------------------------------------------ periodic boxes

int bh_moments_export_trace(bh_ctx *ctx, const bh_moments *m, double *S) {
    int rc = require_gpu(ctx);
    if (rc) return rc;
    if (!m || !S) return fail(ctx, BH_EINVAL, "moments handle or S is NULL");
    const int64_t nn = m->grid->topo.n_nodes;
    HIPX(ctx, hipMemcpyAsync(S, m->d_s, (size_t)nn * sizeof(double), hipMemcpyDeviceToHost, ctx->stream),
         "copy of S");
    HIPX(ctx, hipStreamSynchronize(ctx->stream), "synchronise");
    return BH_OK;
}

int bh_ewald_create(bh_ctx *ctx, double box_size, int n_points, bh_ewald **out) {
    int rc = require_gpu(ctx);
    if (rc) return rc;
    if (!out) return fail(ctx, BH_EINVAL, "output handle pointer is NULL");
    *out = nullptr;
    if (!(box_size > 0.0) || !std::isfinite(box_size)) return fail(ctx, BH_EINVAL, "box_size must be finite and > 0");
    if (n_points < 3 || n_points > BH_EWALD_MAX_POINTS)
        return fail(ctx, BH_EINVAL, "n_points must be in [3, BH_EWALD_MAX_POINTS]");
    bh_ewald *e = new (std::nothrow) bh_ewald();
    if (!e) return fail(ctx, BH_ENOMEM, "host allocation of the table handle");
    e->ctx = ctx;
    e->device = ctx->device;
    e->L = box_size;
    e->n = n_points;
    e->sp = 0.5 * box_size / (n_points - 1);
    const size_t points = (size_t)n_points * n_points * n_points;
    hipError_t err;
    if ((err = dalloc(&e->d_t64, points * bh::kEwaldValues)) != hipSuccess ||
        (err = dalloc(&e->d_t64c, points * bh::kEwaldCompactDoubles)) != hipSuccess ||
        (err = dalloc(&e->d_t32, points * bh::kEwaldCompactFloats)) != hipSuccess ||
        (err = dalloc(&e->d_near, (size_t)bh::kEwaldNearTerms + 1)) != hipSuccess) {
        bh_ewald_destroy(e);
        return hip_fail(ctx, err, "device allocation of the table");
    }
    if ((err = bh::launch_ewald_table(e, ctx->stream)) != hipSuccess) {
        bh_ewald_destroy(e);
        return hip_fail(ctx, err, "table kernel");
    }
    if ((err = bh::fit_ewald_near_series(e, ctx->stream)) != hipSuccess) {
        bh_ewald_destroy(e);
        return hip_fail(ctx, err, "near-origin series");
    }
    *out = e;
    return BH_OK;
}

int bh_ewald_destroy(bh_ewald *e) {
    if (!e) return BH_OK;
    if (e->device >= 0) (void)hipSetDevice(e->device);
    hfree(e->d_t64);
    hfree(e->d_t64c);
    hfree(e->d_t32);
    hfree(e->d_near);
    delete e;
    return BH_OK;
}

int bh_ewald_near_series(bh_ctx *ctx, const bh_ewald *e, double *coeffs, double *radius, double *max_err) {
    int rc = require_gpu(ctx);
    if (rc) return rc;
    if (!e || !coeffs || !radius || !max_err) return fail(ctx, BH_EINVAL, "table handle or an output is NULL");
    for (int k = 0; k < bh::kEwaldNearTerms; k++) coeffs[k] = e->near_coef[k];
    *radius = e->near_radius;
    *max_err = e->near_err;
    return BH_OK;
}

int bh_ewald_set_local_budget(bh_ctx *ctx, bh_ewald *e, double budget, double *h_max) {
    if (!ctx) return BH_EINVAL;
    if (!e) return fail(ctx, BH_EINVAL, "table handle is NULL");
    if (!std::isfinite(budget) || budget < 0.0) return fail(ctx, BH_EINVAL, "budget must be finite and >= 0");
    e->local_budget = budget;
    if (h_max) *h_max = bh::ewald_local_hmax(e, bh::kLocalSpreadNode);
    return BH_OK;
}

int bh_ewald_export(bh_ctx *ctx, const bh_ewald *e, double *values) {
    int rc = require_gpu(ctx);
    if (rc) return rc;
    if (!e || !values) return fail(ctx, BH_EINVAL, "table handle or values is NULL");
    const size_t count = (size_t)e->n * e->n * e->n * bh::kEwaldValues;
    HIPX(ctx, hipMemcpyAsync(values, e->d_t64, count * sizeof(double), hipMemcpyDeviceToHost, ctx->stream),
         "copy of the table");
    HIPX(ctx, hipStreamSynchronize(ctx->stream), "synchronise");
    return BH_OK;
}

namespace {
int check_periodic(bh_ctx *ctx, const bh_grid *g, const bh_moments *m, const bh_ewald *e) {
    if (!g || !m || !e) return fail(ctx, BH_EINVAL, "grid, moments or table is NULL");
    if (m->grid != g) return fail(ctx, BH_ESTATE, "moments belong to another grid");
    if (std::fabs(g->topo.box - e->L) > 1e-12 * e->L)
        return fail(ctx, BH_EINVAL, "the table was made for another box size");
    return BH_OK;
}
}  // namespace

int bh_walk_potential_periodic(bh_ctx *ctx, const bh_grid *g, const bh_moments *m, const bh_ewald *e, double theta,
                               const float *theta_group, int precision, double G, double *phi, int32_t *counts) {
    int rc = require_gpu(ctx);
    if (rc) return rc;
    if ((rc = check_periodic(ctx, g, m, e))) return rc;
    if (!phi) return fail(ctx, BH_EINVAL, "phi_dev is NULL");
    if (precision != BH_FP64 && precision != BH_FP32) return fail(ctx, BH_EINVAL, "precision must be BH_FP64 or BH_FP32");
    if (!theta_group && !(theta > 0.0 && theta <= 1.0)) return fail(ctx, BH_EINVAL, "theta must be in (0, 1]");
    if (!std::isfinite(G)) return fail(ctx, BH_EINVAL, "G must be finite");
    m->walk_epoch++;
    HIPX(ctx, bh::launch_walk_potential_periodic(g, m, e, theta, theta_group, precision, G, phi, counts, ctx->stream),
         "periodic walk + potential kernel");
    return BH_OK;
}

int bh_direct_periodic(bh_ctx *ctx, const bh_grid *g, const bh_moments *m, const bh_ewald *e, const int64_t *targets,
                       int64_t n, double G, double *phi) {
    int rc = require_gpu(ctx);
    if (rc) return rc;
    if ((rc = check_periodic(ctx, g, m, e))) return rc;
    if (n < 0) return fail(ctx, BH_EINVAL, "n_targets must be >= 0");
    if (n > 0 && (!targets || !phi)) return fail(ctx, BH_EINVAL, "targets_dev or phi_dev is NULL");
    if (!std::isfinite(G)) return fail(ctx, BH_EINVAL, "G must be finite");
    HIPX(ctx, bh::launch_direct_periodic(g, m, e, targets, n, G, phi, ctx->stream), "periodic direct-sum kernel");
    return BH_OK;
}

}  // extern "C"
