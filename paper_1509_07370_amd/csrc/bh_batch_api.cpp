// C ABI of the batched path: many grids, one persistent fused launch, optional
// graph capture.  Argument checking, ownership and launch order only.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <new>
#include <numeric>
#include <string>
#include <vector>

#include "bh_internal.h"

struct bh_batch {
    bh_ctx *ctx = nullptr;
    int device = -1;  // for destroy, which does not touch the context
    std::vector<const bh_grid *> grids;
    std::vector<bh_moments *> moments;
    std::vector<int64_t> group_base;      // first queue slot of each grid, size n + 1
    int64_t total = 0;
    bh::WalkArgs *h_desc = nullptr;       // pinned
    bh::WalkArgs *d_desc = nullptr;
    int2 *d_order = nullptr;              // [total] (grid, internal group)
    int32_t *d_counts = nullptr;          // [total][2], per grid in canonical group order
    unsigned long long *d_counter = nullptr;
    int cus = 0;
    int workgroups_per_cu = 0;            // 0: one per resident slot
    int order_mode = BH_ORDER_NATURAL;
    int waves = 0;                        // kernel variant, 0: default of the precision
    int stack_limit = 0;                  // 0: largest safe per grid
    hipStream_t cap_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int precision = BH_FP32;
};

namespace {

int fail(bh_ctx *ctx, int code, const std::string &msg) {
    if (ctx) ctx->err = msg;
    return code;
}

int hip_fail(bh_ctx *ctx, hipError_t e, const char *what) {
    return fail(ctx, e == hipErrorOutOfMemory ? BH_ENOMEM : BH_EDEVICE,
                std::string(what) + ": " + hipGetErrorName(e) + " (" + hipGetErrorString(e) + ")");
}

#define HIPX(ctx, expr, what)                                 \
    do {                                                      \
        hipError_t _e = (expr);                               \
        if (_e != hipSuccess) return hip_fail(ctx, _e, what); \
    } while (0)

int require_gpu(bh_ctx *ctx) {
    if (!ctx) return BH_EINVAL;
    if (ctx->device < 0) return fail(ctx, BH_ESTATE, "host-only context: no GPU work possible");
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return hip_fail(ctx, e, "hipSetDevice");
    return BH_OK;
}

void drop_graph(bh_batch *b) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
}

int upload_order(bh_ctx *ctx, bh_batch *b, const std::vector<int2> &order) {
    HIPX(ctx, hipMemcpy(b->d_order, order.data(), order.size() * sizeof(int2), hipMemcpyHostToDevice), "order");
    return BH_OK;
}

// moments of every grid, then the persistent fused launch, all on stream s; with a table, the periodic walk
int enqueue_solve(bh_ctx *ctx, bh_batch *b, const double *const *rho, double *const *phi, double theta,
                  const float *const *theta_group, int precision, double G, hipStream_t s,
                  const bh_ewald *table = nullptr) {
    const int n = (int)b->grids.size();
    for (int k = 0; k < n; k++) {
        const bh_grid *g = b->grids[k];
        const float *tg = theta_group ? theta_group[k] : nullptr;
        b->h_desc[k] = bh::fused_args(g, b->moments[k], theta, tg, precision, G, phi[k],
                                      b->d_counts + 2 * b->group_base[k], 1);
        if (table) bh::periodic_args(b->h_desc[k], g, b->moments[k], table, precision);
        if (b->stack_limit > 0 && b->stack_limit < b->h_desc[k].k8_threshold)
            b->h_desc[k].k8_threshold = b->stack_limit;
    }
    HIPX(ctx, hipMemcpyAsync(b->d_desc, b->h_desc, n * sizeof(bh::WalkArgs), hipMemcpyHostToDevice, s),
         "upload of the batch descriptors");
    HIPX(ctx, bh::launch_batch_reset(b->d_desc, n, b->d_counter, s), "batch reset kernel");
    for (int k = 0; k < n; k++)
        HIPX(ctx, bh::launch_moments(b->grids[k], b->moments[k], rho[k], s, 1), "moments kernels");
    const bool local = table && b->h_desc[0].ewald_local_hmax > 0.0;
    const int waves = table ? bh::periodic_waves_per_simd(precision, local)
                            : (b->waves > 0 ? b->waves : bh::fused_waves_per_simd(precision));
    int per_cu = b->workgroups_per_cu > 0 ? b->workgroups_per_cu : waves;
    int64_t wgs = (int64_t)b->cus * per_cu;
    const int64_t need = (b->total + 3) / 4;
    if (wgs > need) wgs = need;
    if (wgs < 1) wgs = 1;
    if (table)
        HIPX(ctx, bh::launch_batch_walk_potential_periodic(b->d_desc, b->d_order, b->total, b->d_counter, precision,
                                                           local, (int)wgs, s),
             "batch periodic walk + potential kernel");
    else
        HIPX(ctx, bh::launch_batch_walk_potential(b->d_desc, b->d_order, b->total, b->d_counter, precision, waves,
                                                  (int)wgs, s),
             "batch walk + potential kernel");
    return BH_OK;
}

int check_args(bh_ctx *ctx, bh_batch *b, const double *const *rho, double *const *phi, double theta,
               const float *const *theta_group, int precision, double G) {
    if (!b || !rho || !phi) return fail(ctx, BH_EINVAL, "batch, rho or phi array is NULL");
    if (precision != BH_FP64 && precision != BH_FP32) return fail(ctx, BH_EINVAL, "precision must be BH_FP64 or BH_FP32");
    if (!std::isfinite(G)) return fail(ctx, BH_EINVAL, "G must be finite");
    if (b->waves > 0 && !bh::fused_variant_exists(precision, b->waves))
        return fail(ctx, BH_EINVAL, "waves_per_simd " + std::to_string(b->waves) + " has no " +
                                        (precision == BH_FP64 ? "fp64" : "fp32") + " kernel variant");
    for (size_t k = 0; k < b->grids.size(); k++) {
        if (!rho[k] || !phi[k]) return fail(ctx, BH_EINVAL, "a rho_dev or phi_dev entry is NULL");
        const bool has_tg = theta_group && theta_group[k];
        if (!has_tg && !(theta > 0.0 && theta <= 1.0)) return fail(ctx, BH_EINVAL, "theta must be in (0, 1]");
    }
    return BH_OK;
}

}  // namespace

extern "C" {

int bh_batch_destroy(bh_batch *b) {
    if (!b) return BH_OK;
    if (b->device >= 0) (void)hipSetDevice(b->device);
    drop_graph(b);
    for (auto *m : b->moments) bh_moments_destroy(m);
    if (b->h_desc) (void)hipHostFree(b->h_desc);
    if (b->d_desc) (void)hipFree(b->d_desc);
    if (b->d_order) (void)hipFree(b->d_order);
    if (b->d_counts) (void)hipFree(b->d_counts);
    if (b->d_counter) (void)hipFree(b->d_counter);
    if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
    delete b;
    return BH_OK;
}

int bh_batch_create(bh_ctx *ctx, bh_batch **out, int n, bh_grid *const *grids) {
    int rc = require_gpu(ctx);
    if (rc) return rc;
    if (!out || !grids || n <= 0) return fail(ctx, BH_EINVAL, "batch needs at least one grid");
    *out = nullptr;
    bh_batch *b = new (std::nothrow) bh_batch();
    if (!b) return fail(ctx, BH_ENOMEM, "host allocation of the batch");
    b->ctx = ctx;
    b->device = ctx->device;
    b->group_base.assign(1, 0);
    for (int k = 0; k < n; k++) {
        if (!grids[k] || grids[k]->ctx != ctx) {
            bh_batch_destroy(b);
            return fail(ctx, BH_EINVAL, "a grid is NULL or belongs to another context");
        }
        if (grids[k]->group_cells != bh::kGroupCells) {
            bh_batch_destroy(b);
            return fail(ctx, BH_EINVAL, "batched grids must have 64-cell groups");
        }
        b->grids.push_back(grids[k]);
        b->group_base.push_back(b->group_base.back() + grids[k]->n_groups);
    }
    b->total = b->group_base.back();
    hipDeviceProp_t prop;
    hipError_t e = hipGetDeviceProperties(&prop, ctx->device);
    if (e != hipSuccess) {
        bh_batch_destroy(b);
        return hip_fail(ctx, e, "hipGetDeviceProperties");
    }
    b->cus = prop.multiProcessorCount;
    if ((e = hipHostMalloc((void **)&b->h_desc, n * sizeof(bh::WalkArgs), hipHostMallocDefault)) != hipSuccess ||
        (e = hipMalloc((void **)&b->d_desc, n * sizeof(bh::WalkArgs))) != hipSuccess ||
        (e = hipMalloc((void **)&b->d_order, b->total * sizeof(int2))) != hipSuccess ||
        (e = hipMalloc((void **)&b->d_counts, 2 * b->total * sizeof(int32_t))) != hipSuccess ||
        (e = hipMalloc((void **)&b->d_counter, sizeof(unsigned long long))) != hipSuccess ||
        (e = hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking)) != hipSuccess) {
        bh_batch_destroy(b);
        return hip_fail(ctx, e, "allocation of the batch");
    }
    for (int k = 0; k < n; k++) {
        bh_moments *m = new (std::nothrow) bh_moments();  // batch-owned moments of grid k
        if (!m) {
            bh_batch_destroy(b);
            return fail(ctx, BH_ENOMEM, "host allocation of the moments");
        }
        m->grid = grids[k];
        m->device = ctx->device;
        b->moments.push_back(m);
        const int64_t nn = grids[k]->topo.n_nodes, nc = grids[k]->n_cells;
        if ((e = hipMalloc((void **)&m->d_mom, nn * bh::kMom * sizeof(double))) != hipSuccess ||
            (e = hipMalloc((void **)&m->d_s, nn * sizeof(double))) != hipSuccess ||
            (e = hipMalloc((void **)&m->d_brow, grids[k]->topo.leaves.size() * bh::kBlockRow * sizeof(double))) !=
                hipSuccess ||
            (e = hipMalloc((void **)&m->d_w32, nn * sizeof(bh::WalkRec32))) != hipSuccess ||
            (e = hipMalloc((void **)&m->d_w64, nn * sizeof(bh::WalkRec64))) != hipSuccess ||
            (e = hipMalloc((void **)&m->d_f32, nn * sizeof(bh::FarRec32))) != hipSuccess ||
            (e = hipMalloc((void **)&m->d_cell64, nc * sizeof(double4))) != hipSuccess ||
            (e = hipMalloc((void **)&m->d_cell32, nc * sizeof(float4))) != hipSuccess ||
            (e = hipMalloc((void **)&m->d_flags, 2 * sizeof(int))) != hipSuccess ||
            (e = hipMemset(m->d_flags, 0, 2 * sizeof(int))) != hipSuccess) {
            bh_batch_destroy(b);
            return hip_fail(ctx, e, "allocation of the batch moments");
        }
    }
    std::vector<int2> order(b->total);
    for (int k = 0; k < n; k++)
        for (int64_t q = 0; q < grids[k]->n_groups; q++) order[b->group_base[k] + q] = make_int2(k, (int)q);
    rc = upload_order(ctx, b, order);
    if (rc) {
        bh_batch_destroy(b);
        return rc;
    }
    *out = b;
    return BH_OK;
}

int bh_batch_info(const bh_batch *b, int *n_grids, int64_t *n_groups) {
    if (!b) return BH_EINVAL;
    if (n_grids) *n_grids = (int)b->grids.size();
    if (n_groups) *n_groups = b->total;
    return BH_OK;
}

int bh_batch_set_launch(bh_ctx *ctx, bh_batch *b, int workgroups_per_cu) {
    if (!ctx || !b) return BH_EINVAL;
    if (workgroups_per_cu < 0 || workgroups_per_cu > 64) return fail(ctx, BH_EINVAL, "workgroups_per_cu out of range");
    b->workgroups_per_cu = workgroups_per_cu;
    drop_graph(b);
    return BH_OK;
}

int bh_batch_solve(bh_ctx *ctx, bh_batch *b, const double *const *rho, double *const *phi, double theta,
                   const float *const *theta_group, int precision, double G) {
    int rc = require_gpu(ctx);
    if (rc) return rc;
    if ((rc = check_args(ctx, b, rho, phi, theta, theta_group, precision, G))) return rc;
    b->precision = precision;
    return enqueue_solve(ctx, b, rho, phi, theta, theta_group, precision, G, ctx->stream);
}

int bh_batch_solve_periodic(bh_ctx *ctx, bh_batch *b, const bh_ewald *table, const double *const *rho,
                            double *const *phi, double theta, const float *const *theta_group, int precision,
                            double G) {
    int rc = require_gpu(ctx);
    if (rc) return rc;
    if (!table) return fail(ctx, BH_EINVAL, "table handle is NULL");
    if ((rc = check_args(ctx, b, rho, phi, theta, theta_group, precision, G))) return rc;
    if (table->device != ctx->device) return fail(ctx, BH_EDEVICE, "the table lives on another device");
    for (const bh_grid *g : b->grids)
        if (std::fabs(g->topo.box - table->L) > 1e-12 * table->L)
            return fail(ctx, BH_EINVAL, "every grid's box must be the table's");
    b->precision = precision;
    return enqueue_solve(ctx, b, rho, phi, theta, theta_group, precision, G, ctx->stream, table);
}

int bh_batch_capture(bh_ctx *ctx, bh_batch *b, const double *const *rho, double *const *phi, double theta,
                     const float *const *theta_group, int precision, double G) {
    int rc = require_gpu(ctx);
    if (rc) return rc;
    if ((rc = check_args(ctx, b, rho, phi, theta, theta_group, precision, G))) return rc;
    drop_graph(b);
    b->precision = precision;
    HIPX(ctx, hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal), "begin capture");
    rc = enqueue_solve(ctx, b, rho, phi, theta, theta_group, precision, G, b->cap_stream);
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamEndCapture(b->cap_stream, &graph);
    if (rc) {
        if (graph) (void)hipGraphDestroy(graph);
        return rc;
    }
    if (e != hipSuccess) return hip_fail(ctx, e, "end capture");
    b->graph = graph;
    HIPX(ctx, hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0), "graph instantiation");
    return BH_OK;
}

int bh_batch_replay(bh_ctx *ctx, bh_batch *b) {
    int rc = require_gpu(ctx);
    if (rc) return rc;
    if (!b || !b->exec) return fail(ctx, BH_ESTATE, "no captured graph (call bh_batch_capture first)");
    HIPX(ctx, hipGraphLaunch(b->exec, ctx->stream), "graph launch");
    return BH_OK;
}

int bh_batch_check(bh_ctx *ctx, const bh_batch *b) {
    int rc = require_gpu(ctx);
    if (rc) return rc;
    if (!b) return fail(ctx, BH_EINVAL, "batch is NULL");
    std::vector<int> flags(2 * b->grids.size());
    for (size_t k = 0; k < b->grids.size(); k++)
        HIPX(ctx, hipMemcpyAsync(&flags[2 * k], b->moments[k]->d_flags, 2 * sizeof(int), hipMemcpyDeviceToHost,
                                 ctx->stream), "copy flags");
    HIPX(ctx, hipStreamSynchronize(ctx->stream), "synchronise");
    for (size_t k = 0; k < b->grids.size(); k++) {
        if (flags[2 * k]) return fail(ctx, BH_EINVAL, "grid " + std::to_string(k) + ": densities must be finite and >= 0");
        if (flags[2 * k + 1]) return fail(ctx, BH_ECAPACITY, "grid " + std::to_string(k) + ": walk stack overflow");
    }
    return BH_OK;
}

int bh_batch_counts(bh_ctx *ctx, const bh_batch *b, int32_t *counts) {
    int rc = require_gpu(ctx);
    if (rc) return rc;
    if (!b || !counts) return fail(ctx, BH_EINVAL, "batch or counts is NULL");
    HIPX(ctx, hipMemcpyAsync(counts, b->d_counts, 2 * b->total * sizeof(int32_t), hipMemcpyDeviceToHost, ctx->stream),
         "copy counts");
    HIPX(ctx, hipStreamSynchronize(ctx->stream), "synchronise");
    return BH_OK;
}

int bh_batch_schedule(bh_ctx *ctx, bh_batch *b, int mode) {
    int rc = require_gpu(ctx);
    if (rc) return rc;
    if (!b) return fail(ctx, BH_EINVAL, "batch is NULL");
    if (mode != BH_ORDER_NATURAL && mode != BH_ORDER_COST) return fail(ctx, BH_EINVAL, "unknown schedule mode");
    const int n = (int)b->grids.size();
    std::vector<int2> order(b->total);
    for (int k = 0; k < n; k++)
        for (int64_t q = 0; q < b->grids[k]->n_groups; q++) order[b->group_base[k] + q] = make_int2(k, (int)q);
    if (mode == BH_ORDER_COST) {
        std::vector<int32_t> c(2 * b->total);
        rc = bh_batch_counts(ctx, b, c.data());
        if (rc) return rc;
        // counts are stored per grid in canonical group order; queue items name internal groups
        std::vector<double> cost(b->total);
        for (int k = 0; k < n; k++) {
            const bh_grid *g = b->grids[k];
            const int per = bh::kCellsPerBlock / g->group_cells;
            for (int64_t q = 0; q < g->n_groups; q++) {
                const int64_t cg = (int64_t)g->topo.leaves[q / per].canon * per + q % per;
                const int64_t i = b->group_base[k] + cg;
                cost[b->group_base[k] + q] = 35.0 * 64 * c[2 * i] + 11.0 * (512.0 * c[2 * i + 1] - 64);
            }
        }
        std::vector<int64_t> idx(b->total);
        std::iota(idx.begin(), idx.end(), 0);
        std::stable_sort(idx.begin(), idx.end(), [&](int64_t x, int64_t y) { return cost[x] > cost[y]; });
        std::vector<int2> sorted(b->total);
        for (int64_t i = 0; i < b->total; i++) sorted[i] = order[idx[i]];
        order.swap(sorted);
    }
    drop_graph(b);
    rc = upload_order(ctx, b, order);
    if (rc == BH_OK) b->order_mode = mode;
    return rc;
}

int bh_batch_get_config(const bh_batch *b, bh_batch_config *cfg) {
    if (!b || !cfg) return BH_EINVAL;
    cfg->order = b->order_mode;
    cfg->workgroups_per_cu = b->workgroups_per_cu;
    cfg->waves_per_simd = b->waves;
    cfg->stack_limit = b->stack_limit;
    return BH_OK;
}

int bh_batch_configure(bh_ctx *ctx, bh_batch *b, const bh_batch_config *cfg) {
    if (!ctx || !b || !cfg) return fail(ctx, BH_EINVAL, "context, batch or config is NULL");
    if (cfg->order != BH_ORDER_NATURAL && cfg->order != BH_ORDER_COST)
        return fail(ctx, BH_EINVAL, "unknown queue order");
    if (cfg->workgroups_per_cu < 0 || cfg->workgroups_per_cu > 64)
        return fail(ctx, BH_EINVAL, "workgroups_per_cu out of range");
    if (cfg->waves_per_simd != 0 && !bh::fused_variant_exists(BH_FP32, cfg->waves_per_simd) &&
        !bh::fused_variant_exists(BH_FP64, cfg->waves_per_simd))
        return fail(ctx, BH_EINVAL, "no kernel variant for waves_per_simd " + std::to_string(cfg->waves_per_simd));
    if (cfg->stack_limit != 0 && (cfg->stack_limit < 8 || cfg->stack_limit > bh::kWalkStackCap))
        return fail(ctx, BH_EINVAL, "stack_limit must be 0 or in [8, stack capacity]");
    int rc = bh_batch_schedule(ctx, b, cfg->order);
    if (rc) return rc;
    b->workgroups_per_cu = cfg->workgroups_per_cu;
    b->waves = cfg->waves_per_simd;
    b->stack_limit = cfg->stack_limit;
    drop_graph(b);
    return BH_OK;
}

int bh_batch_autotune(bh_ctx *ctx, bh_batch *b, const double *const *rho, double *const *phi, double theta,
                      const float *const *theta_group, int precision, double G, int reps, bh_batch_config *best,
                      float *best_ms, bh_batch_timing *table, int table_cap, int *n_table) {
    int rc = require_gpu(ctx);
    if (rc) return rc;
    if (!b) return fail(ctx, BH_EINVAL, "batch is NULL");
    if (reps < 1) return fail(ctx, BH_EINVAL, "reps must be >= 1");
    if (table_cap < 0 || (table_cap > 0 && !table)) return fail(ctx, BH_EINVAL, "table is NULL or table_cap < 0");
    const bh_batch_config saved = {b->order_mode, b->workgroups_per_cu, b->waves, b->stack_limit};
    b->waves = 0;
    if ((rc = check_args(ctx, b, rho, phi, theta, theta_group, precision, G))) return rc;
    drop_graph(b);
    // a first solve fills the counts that the cost order needs
    b->precision = precision;
    if ((rc = enqueue_solve(ctx, b, rho, phi, theta, theta_group, precision, G, ctx->stream))) return rc;
    std::vector<bh_batch_config> cands;
    const int variants32[] = {8, 6, 4}, variants64[] = {4, 2};
    const int *var = precision == BH_FP64 ? variants64 : variants32;
    const int nvar = precision == BH_FP64 ? 2 : 3;
    for (int order : {BH_ORDER_NATURAL, BH_ORDER_COST})
        for (int v = 0; v < nvar; v++) {
            std::vector<int> widths = {var[v], var[v] / 2, 1};
            std::sort(widths.begin(), widths.end());
            widths.erase(std::unique(widths.begin(), widths.end()), widths.end());
            for (int w : widths)
                for (int stack : {0, 64}) cands.push_back({order, w, var[v], stack});
        }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIPX(ctx, hipEventCreate(&e0), "event");
    hipError_t he = hipEventCreate(&e1);
    if (he != hipSuccess) {
        (void)hipEventDestroy(e0);
        return hip_fail(ctx, he, "event");
    }
    std::vector<float> med(cands.size(), 0.f);
    int best_i = -1;
    for (size_t c = 0; c < cands.size() && rc == BH_OK; c++) {
        if (c == 0 || cands[c].order != cands[c - 1].order) rc = bh_batch_schedule(ctx, b, cands[c].order);
        if (rc) break;
        b->workgroups_per_cu = cands[c].workgroups_per_cu;
        b->waves = cands[c].waves_per_simd;
        b->stack_limit = cands[c].stack_limit;
        if ((rc = enqueue_solve(ctx, b, rho, phi, theta, theta_group, precision, G, ctx->stream))) break;
        std::vector<float> t(reps);
        for (int r = 0; r < reps && rc == BH_OK; r++) {
            if ((he = hipEventRecord(e0, ctx->stream)) != hipSuccess) { rc = hip_fail(ctx, he, "event record"); break; }
            if ((rc = enqueue_solve(ctx, b, rho, phi, theta, theta_group, precision, G, ctx->stream))) break;
            if ((he = hipEventRecord(e1, ctx->stream)) != hipSuccess ||
                (he = hipEventSynchronize(e1)) != hipSuccess || (he = hipEventElapsedTime(&t[r], e0, e1)) != hipSuccess)
                rc = hip_fail(ctx, he, "event timing");
        }
        if (rc) break;
        std::sort(t.begin(), t.end());
        med[c] = t[reps / 2];
        if (best_i < 0 || med[c] < med[best_i]) best_i = (int)c;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) {  // leave the batch as it was
        b->workgroups_per_cu = saved.workgroups_per_cu;
        b->waves = saved.waves_per_simd;
        b->stack_limit = saved.stack_limit;
        (void)bh_batch_schedule(ctx, b, saved.order);
        return rc;
    }
    const bh_batch_config &w = cands[best_i];
    if ((rc = bh_batch_configure(ctx, b, &w))) return rc;
    if (best) *best = w;
    if (best_ms) *best_ms = med[best_i];
    for (int c = 0; c < (int)cands.size() && c < table_cap; c++) table[c] = {cands[c], med[c]};
    if (n_table) *n_table = (int)cands.size();
    return BH_OK;
}

}  // extern "C"
