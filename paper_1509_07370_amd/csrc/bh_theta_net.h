// The per-group opening-angle network evaluated by one wavefront: group
// features from node rows, then the bf16 network 12 -> 64 -> 64 -> 1 with one
// hidden unit per lane.  Shared by the stand-alone inference kernel and the
// walk kernel that infers each group's theta before walking it, so that both
// produce the same theta bit for bit.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "bh.h"
#include "bh_device.h"
#include "bh_internal.h"

namespace bh {

// parameter layout (fp32 and bf16 copies): W1[64][12], b1[64], W2[64][64], b2[64], w3[64], b3
constexpr int OW1 = 0, OB1 = 768, OW2 = 832, OB2 = 4928, OW3 = 4992, OB3 = 5056;

__device__ __forceinline__ float bf16_round(float x) {
    uint32_t u = __float_as_uint(x);
    u = (u + 0x7FFFu + ((u >> 16) & 1u)) & 0xFFFF0000u;  // round to nearest even
    return __uint_as_float(u);
}
__device__ __forceinline__ float bf16_load(const uint16_t *p, int i) { return __uint_as_float((uint32_t)p[i] << 16); }

__device__ __forceinline__ float wave_sum(float v) {
    // fixed butterfly order: deterministic, every lane ends with the same bits
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ double log_floor(double x, double floor) { return log(x > floor ? x : floor); }

// Everything the network needs besides the group: parameters and the grid's
// node rows (moments slot 11 = the group node's largest cell mass).
struct ThetaNetArgs {
    const uint16_t *w;  // bf16 parameters, layout above (16-byte aligned)
    const float *mean, *scale;
    float shift;
    const double *mom;
    const double *geom;
    const int32_t *parent;
    int root;
    int nbase;
    double box;
};

// theta of group (L, sub) on one wavefront; xs: 12 floats, hs: 64 floats of
// this wavefront's LDS.  Feature order as in the features kernel.
__device__ inline float group_theta(const ThetaNetArgs &n, const LeafInfo &L, int sub, int lane,
                                                      float *xs, float *hs) {
    // this lane's weights first, all loads independent: W1 row (12 bf16 as
    // three 8-byte loads), W2 row (64 bf16 as eight 16-byte loads), biases
    const uint2 *r1 = reinterpret_cast<const uint2 *>(n.w + OW1 + lane * BH_MLP_INPUTS);
    const uint4 *r2 = reinterpret_cast<const uint4 *>(n.w + OW2 + lane * BH_MLP_HIDDEN);
    uint2 w1[3];
    uint4 w2[8];
#pragma unroll
    for (int q = 0; q < 3; q++) w1[q] = r1[q];
#pragma unroll
    for (int q = 0; q < 8; q++) w2[q] = r2[q];
    const float b1 = bf16_load(n.w, OB1 + lane), b2 = bf16_load(n.w, OB2 + lane);
    const float w3 = bf16_load(n.w, OW3 + lane), b3 = bf16_load(n.w, OB3);
    const float mu = lane < BH_MLP_INPUTS ? n.mean[lane] : 0.0f, sc = lane < BH_MLP_INPUTS ? n.scale[lane] : 0.0f;
    // lane i < 12 derives feature i: its argument in fp64 from the node rows,
    // then one fp32 logarithm (order as in the features kernel)
    const int gnode = L.oct_first + sub;
    if (lane < BH_MLP_INPUTS) {
        float f = 6.0f;  // 0: log2(group cells)
        if (lane == 1 || lane == 4 || lane == 11) {
            const double Mg = n.mom[(int64_t)gnode * kMom + 3];
            if (lane == 1) {
                const double Mroot = n.mom[(int64_t)n.root * kMom + 3];
                const double r = Mroot > 0.0 ? Mg / Mroot : 0.0;
                f = logf((float)(r > 1e-30 ? r : 1e-30));
            } else if (lane == 4) {
                const double mmax = n.mom[(int64_t)gnode * kMom + 11];
                f = Mg > 0.0 ? logf((float)(mmax / (Mg / 64.0))) : 0.0f;
            } else {
                const double Mb = n.mom[(int64_t)L.block_node * kMom + 3];
                const double r = Mb > 0.0 ? 8.0 * Mg / Mb : 0.0;
                f = Mb > 0.0 ? logf((float)(r > 1e-30 ? r : 1e-30)) : 0.0f;
            }
        } else if (lane == 2) {
            f = logf((float)(4.0 * L.h / n.box));
        } else if (lane == 3) {
            f = rintf(log2f((float)(n.box / ((double)n.nbase * kNB * L.h))));
        } else if (lane >= 5) {  // 5..10: (delta/l, |Q|/(M l^2)) of group node, block, block's parent
            const int a = (lane - 5) >> 1;
            const int pn = n.parent[L.block_node];
            const int node = a == 0 ? gnode : (a == 1 ? L.block_node : (pn >= 0 ? pn : L.block_node));
            const double *r = n.mom + (int64_t)node * kMom;
            const double l = n.geom[4 * (int64_t)node + 3];
            double arg;
            if (((lane - 5) & 1) == 0) {
                arg = r[10] / l + 1e-6;
            } else {
                const double M = r[3];
                const double qf =
                    sqrt(r[4] * r[4] + r[5] * r[5] + r[6] * r[6] + 2.0 * (r[7] * r[7] + r[8] * r[8] + r[9] * r[9]));
                arg = (M > 0.0 ? qf / (M * l * l) : 0.0) + 1e-6;
            }
            f = logf((float)arg);
        }
        xs[lane] = f;
    }
    wave_lds_sync();
    if (lane < BH_MLP_INPUTS) xs[lane] = bf16_round((xs[lane] - mu) * sc);
    wave_lds_sync();
    float a1 = b1;
#pragma unroll
    for (int q = 0; q < 3; q++) {
        const uint32_t wv[2] = {w1[q].x, w1[q].y};
#pragma unroll
        for (int p = 0; p < 2; p++) {
            a1 = fmaf(__uint_as_float(wv[p] << 16), xs[4 * q + 2 * p], a1);
            a1 = fmaf(__uint_as_float(wv[p] & 0xFFFF0000u), xs[4 * q + 2 * p + 1], a1);
        }
    }
    hs[lane] = bf16_round(tanhf(a1));
    wave_lds_sync();
    float a2 = b2;
#pragma unroll
    for (int k8 = 0; k8 < BH_MLP_HIDDEN / 8; k8++) {
        const uint32_t wv[4] = {w2[k8].x, w2[k8].y, w2[k8].z, w2[k8].w};
#pragma unroll
        for (int p = 0; p < 4; p++) {
            a2 = fmaf(__uint_as_float(wv[p] << 16), hs[8 * k8 + 2 * p], a2);
            a2 = fmaf(__uint_as_float(wv[p] & 0xFFFF0000u), hs[8 * k8 + 2 * p + 1], a2);
        }
    }
    const float z = wave_sum(w3 * bf16_round(tanhf(a2))) + b3;
    wave_lds_sync();  // xs / hs may be reused by the caller
    const float th = 0.2f + 0.8f / (1.0f + expf(-z)) - n.shift;
    // snapped up to the grid 0.20, 0.25, ..., 1.00 on which the labels and the
    // safety shift are defined (the shift is calibrated charging each
    // prediction the error of the next grid value up): the walk then uses a
    // value whose error was measured, and a network saturating just below 1
    // walks at 1
    int k = (int)ceilf((th - 1e-6f - 0.2f) * 20.0f);
    k = k < 0 ? 0 : (k > 16 ? 16 : k);
    return (float)(0.2 + 0.05 * (double)k);
}

}  // namespace bh
