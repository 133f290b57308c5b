// Internal declarations of the learned-theta part (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "bh.h"
#include "bh_internal.h"
#include "bh_theta_net.h"

namespace bh {
constexpr int kMlpIn = BH_MLP_INPUTS;
constexpr int kMlpHidden = BH_MLP_HIDDEN;
constexpr int kMlpParams = BH_MLP_PARAMS;
constexpr int kMlpChunks = 256;  // partial gradients per gradient evaluation

hipError_t launch_features(const bh_grid *g, const bh_moments *m, float *out, hipStream_t s);
hipError_t launch_group_rms(const bh_grid *g, const double *phi, const double *ref, float *out, hipStream_t s);
}  // namespace bh

struct bh_mlp {
    bh_ctx *ctx = nullptr;
    int device = -1;  // for destroy, which does not touch the context
    float *d_params = nullptr;   // [kMlpParams]
    uint16_t *d_bf16 = nullptr;  // bf16 copy of the parameters
    float *d_mean = nullptr, *d_scale = nullptr;  // [kMlpIn]
    float *d_m = nullptr, *d_v = nullptr;         // Adam moments
    float *d_partials = nullptr;                  // [kMlpChunks][kMlpParams + 1]
    int step = 0;
    int theta_floor_k = 0;  // inference never returns a theta below 0.20 + 0.05 * theta_floor_k
};

namespace bh {
hipError_t launch_mlp_bf16(bh_mlp *net, hipStream_t s);
ThetaNetArgs theta_net_args(const bh_grid *g, const bh_moments *m, const bh_mlp *net, float shift);
hipError_t launch_theta_infer(const bh_grid *g, const bh_moments *m, const bh_mlp *net, float shift, float *theta,
                              hipStream_t s);
hipError_t launch_mlp_forward(const bh_mlp *net, const float *feat, int64_t n, bool bf16, float shift, float *theta,
                              hipStream_t s);
hipError_t launch_mlp_grad(bh_mlp *net, const float *feat, const float *label, int64_t n, float *grad, float *loss,
                           hipStream_t s);
hipError_t launch_mlp_adam(bh_mlp *net, const float *grad, float lr, float b1, float b2, float eps, hipStream_t s);
}  // namespace bh
