// C ABI of the learned-theta part: argument checking and ownership only.
#include <hip/hip_runtime.h>

#include <cmath>
#include <new>
#include <string>

#include "bh_internal.h"
#include "bh_mlp.h"

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

void hfree(void *p) {
    if (p) (void)hipFree(p);
}

}  // namespace

extern "C" {

int bh_group_features(bh_ctx *ctx, const bh_grid *g, const bh_moments *m, float *feat) {
    int rc = require_gpu(ctx);
    if (rc) return rc;
    if (!g || !m || !feat) return fail(ctx, BH_EINVAL, "grid, moments or feat_dev is NULL");
    if (m->grid != g) return fail(ctx, BH_ESTATE, "moments were built for another grid");
    if (g->group_cells != bh::kGroupCells) return fail(ctx, BH_EINVAL, "the network's features need 64-cell groups");
    HIPX(ctx, bh::launch_features(g, m, feat, ctx->stream), "features kernel");
    return BH_OK;
}

int bh_group_rms_error(bh_ctx *ctx, const bh_grid *g, const double *phi, const double *ref, float *rms) {
    int rc = require_gpu(ctx);
    if (rc) return rc;
    if (!g || !phi || !ref || !rms) return fail(ctx, BH_EINVAL, "grid, phi_dev, ref_dev or rms_dev is NULL");
    if (g->group_cells != bh::kGroupCells) return fail(ctx, BH_EINVAL, "per-group errors need 64-cell groups");
    HIPX(ctx, bh::launch_group_rms(g, phi, ref, rms, ctx->stream), "group error kernel");
    return BH_OK;
}

int bh_mlp_destroy(bh_mlp *net) {
    if (!net) return BH_OK;
    if (net->device >= 0) (void)hipSetDevice(net->device);
    hfree(net->d_params);
    hfree(net->d_bf16);
    hfree(net->d_mean);
    hfree(net->d_scale);
    hfree(net->d_m);
    hfree(net->d_v);
    hfree(net->d_partials);
    delete net;
    return BH_OK;
}

int bh_mlp_create(bh_ctx *ctx, bh_mlp **out, const float *params, const float *mean, const float *scale) {
    int rc = require_gpu(ctx);
    if (rc) return rc;
    if (!out || !params || !mean || !scale) return fail(ctx, BH_EINVAL, "a bh_mlp_create argument is NULL");
    for (int i = 0; i < bh::kMlpParams; i++)
        if (!std::isfinite(params[i])) return fail(ctx, BH_EINVAL, "parameters must be finite");
    for (int i = 0; i < bh::kMlpIn; i++)
        if (!std::isfinite(mean[i]) || !std::isfinite(scale[i]))
            return fail(ctx, BH_EINVAL, "normalisation must be finite");
    bh_mlp *n = new (std::nothrow) bh_mlp();
    if (!n) return fail(ctx, BH_ENOMEM, "host allocation of the network");
    n->ctx = ctx;
    n->device = ctx->device;
    const size_t P = bh::kMlpParams;
    hipError_t e;
    if ((e = hipMalloc((void **)&n->d_params, P * sizeof(float))) != hipSuccess ||
        (e = hipMalloc((void **)&n->d_bf16, P * sizeof(uint16_t))) != hipSuccess ||
        (e = hipMalloc((void **)&n->d_mean, bh::kMlpIn * sizeof(float))) != hipSuccess ||
        (e = hipMalloc((void **)&n->d_scale, bh::kMlpIn * sizeof(float))) != hipSuccess ||
        (e = hipMalloc((void **)&n->d_m, P * sizeof(float))) != hipSuccess ||
        (e = hipMalloc((void **)&n->d_v, P * sizeof(float))) != hipSuccess ||
        (e = hipMalloc((void **)&n->d_partials, (size_t)bh::kMlpChunks * (P + 1) * sizeof(float))) != hipSuccess ||
        (e = hipMemcpy(n->d_params, params, P * sizeof(float), hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(n->d_mean, mean, bh::kMlpIn * sizeof(float), hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(n->d_scale, scale, bh::kMlpIn * sizeof(float), hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemset(n->d_m, 0, P * sizeof(float))) != hipSuccess ||
        (e = hipMemset(n->d_v, 0, P * sizeof(float))) != hipSuccess ||
        (e = bh::launch_mlp_bf16(n, ctx->stream)) != hipSuccess) {
        bh_mlp_destroy(n);
        return hip_fail(ctx, e, "allocation of the network");
    }
    *out = n;
    return BH_OK;
}

int bh_mlp_set_params(bh_ctx *ctx, bh_mlp *net, const float *params) {
    int rc = require_gpu(ctx);
    if (rc) return rc;
    if (!net || !params) return fail(ctx, BH_EINVAL, "network or parameters NULL");
    HIPX(ctx, hipMemcpyAsync(net->d_params, params, bh::kMlpParams * sizeof(float), hipMemcpyHostToDevice, ctx->stream),
         "upload of the parameters");
    HIPX(ctx, bh::launch_mlp_bf16(net, ctx->stream), "bf16 copy");
    HIPX(ctx, hipStreamSynchronize(ctx->stream), "synchronise");
    return BH_OK;
}

int bh_mlp_set_theta_floor(bh_ctx *ctx, bh_mlp *net, float theta_floor) {
    if (!ctx) return BH_EINVAL;
    if (!net) return fail(ctx, BH_EINVAL, "network NULL");
    if (!std::isfinite(theta_floor) || theta_floor < 0.2f || theta_floor > 1.0f)
        return fail(ctx, BH_EINVAL, "theta_floor must lie in [0.2, 1]");
    // the same snap as the inference: up to the next grid value, a value on the grid kept
    const int k = (int)std::ceil((theta_floor - 1e-6f - 0.2f) * 20.0f);
    net->theta_floor_k = k < 0 ? 0 : (k > 16 ? 16 : k);
    return BH_OK;
}

int bh_mlp_get_params(bh_ctx *ctx, const bh_mlp *net, float *params) {
    int rc = require_gpu(ctx);
    if (rc) return rc;
    if (!net || !params) return fail(ctx, BH_EINVAL, "network or parameters NULL");
    HIPX(ctx, hipMemcpyAsync(params, net->d_params, bh::kMlpParams * sizeof(float), hipMemcpyDeviceToHost, ctx->stream),
         "copy of the parameters");
    HIPX(ctx, hipStreamSynchronize(ctx->stream), "synchronise");
    return BH_OK;
}

int bh_mlp_forward(bh_ctx *ctx, const bh_mlp *net, const float *feat, int64_t n, int bf16, float theta_shift,
                   float *theta) {
    int rc = require_gpu(ctx);
    if (rc) return rc;
    if (!net) return fail(ctx, BH_EINVAL, "network is NULL");
    if (n < 0) return fail(ctx, BH_EINVAL, "n must be >= 0");
    if (n > 0 && (!feat || !theta)) return fail(ctx, BH_EINVAL, "feat_dev or theta_dev is NULL");
    if (!std::isfinite(theta_shift)) return fail(ctx, BH_EINVAL, "theta_shift must be finite");
    HIPX(ctx, bh::launch_mlp_forward(net, feat, n, bf16 != 0, theta_shift, theta, ctx->stream),
         "network forward kernel");
    return BH_OK;
}

int bh_learned_walk_potential(bh_ctx *ctx, const bh_grid *g, const bh_moments *m, const bh_mlp *net, float shift,
                              int precision, double G, double *phi, float *theta, int32_t *counts) {
    int rc = require_gpu(ctx);
    if (rc) return rc;
    if (!g || !m || !net || !phi) return fail(ctx, BH_EINVAL, "grid, moments, network or phi_dev is NULL");
    if (m->grid != g) return fail(ctx, BH_ESTATE, "moments were built for another grid");
    if (g->group_cells != bh::kGroupCells) return fail(ctx, BH_EINVAL, "the network's features need 64-cell groups");
    if (precision != BH_FP64 && precision != BH_FP32) return fail(ctx, BH_EINVAL, "precision must be BH_FP64 or BH_FP32");
    if (!std::isfinite(shift)) return fail(ctx, BH_EINVAL, "theta_shift must be finite");
    if (!std::isfinite(G)) return fail(ctx, BH_EINVAL, "G must be finite");
    m->walk_epoch++;
    float *th = theta ? theta : m->d_theta;
    HIPX(ctx, bh::launch_theta_infer(g, m, net, shift, th, ctx->stream), "theta inference kernel");
    HIPX(ctx, bh::launch_walk_potential_theta(g, m, th, precision, G, phi, counts, ctx->stream),
         "walk + potential kernel");
    return BH_OK;
}

int bh_theta_infer(bh_ctx *ctx, const bh_grid *g, const bh_moments *m, const bh_mlp *net, float shift,
                   float *theta) {
    int rc = require_gpu(ctx);
    if (rc) return rc;
    if (!g || !m || !net || !theta) return fail(ctx, BH_EINVAL, "grid, moments, network or theta_dev is NULL");
    if (m->grid != g) return fail(ctx, BH_ESTATE, "moments were built for another grid");
    if (g->group_cells != bh::kGroupCells) return fail(ctx, BH_EINVAL, "the network's features need 64-cell groups");
    if (!std::isfinite(shift)) return fail(ctx, BH_EINVAL, "theta_shift must be finite");
    HIPX(ctx, bh::launch_theta_infer(g, m, net, shift, theta, ctx->stream), "theta inference kernel");
    return BH_OK;
}

int bh_mlp_grad(bh_ctx *ctx, bh_mlp *net, const float *feat, const float *label, int64_t n, float *grad,
                float *loss) {
    int rc = require_gpu(ctx);
    if (rc) return rc;
    if (!net || !feat || !label || !grad) return fail(ctx, BH_EINVAL, "a bh_mlp_grad argument is NULL");
    if (n <= 0) return fail(ctx, BH_EINVAL, "n must be > 0");
    HIPX(ctx, bh::launch_mlp_grad(net, feat, label, n, grad, loss, ctx->stream), "network gradient kernels");
    return BH_OK;
}

int bh_mlp_adam_step(bh_ctx *ctx, bh_mlp *net, const float *grad, float lr, float b1, float b2, float eps) {
    int rc = require_gpu(ctx);
    if (rc) return rc;
    if (!net || !grad) return fail(ctx, BH_EINVAL, "network or grad_dev is NULL");
    if (!(lr > 0.f) || !(b1 >= 0.f && b1 < 1.f) || !(b2 >= 0.f && b2 < 1.f) || !(eps > 0.f))
        return fail(ctx, BH_EINVAL, "Adam hyper-parameters out of range");
    HIPX(ctx, bh::launch_mlp_adam(net, grad, lr, b1, b2, eps, ctx->stream), "Adam kernel");
    return BH_OK;
}

}  // extern "C"
