// The per-group opening-angle network evaluated by one wavefront for up to 16
// groups: group features from node rows, then the bf16 network
// 12 -> 64 -> 64 -> 1 on the matrix cores.
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
    int kmin;  // smallest index on the grid 0.20 + 0.05 k the snapped theta may take
    const double *mom;
    const double *geom;
    const int32_t *leaf_parent;  // [n_leaf] parent node of the leaf block's node (the node itself at the root)
    int root;
    int nbase;
    double box;
};

// The 12 features of group (L, sub): each argument in fp64 from the node rows,
// then one fp32 logarithm (order as in the features kernel).  No branch
// depends on the feature index, so every lane of a wavefront issues the same
// loads (the group's, block's and block parent's node rows) together; the
// parent's id comes from a leaf-indexed array, loaded beside the leaf record.
__device__ __forceinline__ void group_features12(const ThetaNetArgs &n, const LeafInfo &L, int leaf, int sub,
                                                 float *f) {
    const int gnode = L.oct_first + sub;
    const int node[3] = {gnode, L.block_node, n.leaf_parent[leaf]};
    const double Mg = n.mom[(int64_t)gnode * kMom + 3];
    const double Mroot = n.mom[(int64_t)n.root * kMom + 3];
    const double mmax = n.mom[(int64_t)gnode * kMom + 11];
    const double Mb = n.mom[(int64_t)L.block_node * kMom + 3];
    f[0] = 6.0f;  // log2(group cells)
    {
        const double r = Mroot > 0.0 ? Mg / Mroot : 0.0;
        f[1] = logf((float)(r > 1e-30 ? r : 1e-30));
    }
    f[2] = logf((float)(4.0 * L.h / n.box));
    f[3] = rintf(log2f((float)(n.box / ((double)n.nbase * kNB * L.h))));
    f[4] = Mg > 0.0 ? logf((float)(mmax / (Mg / 64.0))) : 0.0f;
#pragma unroll
    for (int a = 0; a < 3; a++) {  // (delta/l, |Q|/(M l^2)) of group node, block, block's parent
        const double *r = n.mom + (int64_t)node[a] * kMom;
        const double l = n.geom[4 * (int64_t)node[a] + 3];
        f[5 + 2 * a] = logf((float)(r[10] / l + 1e-6));
        const double M = r[3];
        const double qf =
            sqrt(r[4] * r[4] + r[5] * r[5] + r[6] * r[6] + 2.0 * (r[7] * r[7] + r[8] * r[8] + r[9] * r[9]));
        f[6 + 2 * a] = logf((float)((M > 0.0 ? qf / (M * l * l) : 0.0) + 1e-6));
    }
    {
        const double r = Mb > 0.0 ? 8.0 * Mg / Mb : 0.0;
        f[11] = Mb > 0.0 ? logf((float)(r > 1e-30 ? r : 1e-30)) : 0.0f;
    }
}

// theta of up to 16 groups g0 .. g0 + cnt - 1 on one wavefront, the network
// as three small matrix products on the matrix cores
// (v_mfma_f32_16x16x16_bf16: bf16 operands, fp32 accumulation).  Lane
// l = c + 16 q (c = l & 15, q = l >> 4) takes part in every product as
// column c and k-slot q (items 0..3 of its operand), and receives rows
// 4q .. 4q + 3 of column c of the result.  The products are written
// transposed, hidden unit x group, so that a layer's result is already in
// the operand layout of the next one: no data moves between lanes.
//   layer 1: H1 (64 x 16) = W1 (64 x 12) X^T (12 x 16) + b1, four row tiles,
//            the 12 inputs packed as k = 3q + i (i < 3; item 3 is zero);
//   layer 2: H2 = W2 (64 x 64) tanh(H1) + b2, k-step s = row tile s of H1;
//   output:  z = w3 . tanh(H2) + b3, per lane over its 16 rows, then across
//            the four lanes of a column in a fixed order.
// The order of the k sum inside a product is the hardware's; results equal
// the fused-multiply-add forward up to fp32 rounding.  Returns group c's
// theta (snapped) in every lane of column c; columns c >= cnt are not valid.
typedef short bh_bf16x4 __attribute__((ext_vector_type(4)));
typedef float bh_f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ short bf16_bits(float x) { return (short)(__float_as_uint(bf16_round(x)) >> 16); }

__device__ inline float groups_theta16(const ThetaNetArgs &n, const LeafInfo *leaves, int64_t g0, int cnt, int lane) {
    const int c = lane & 15, q = lane >> 4;
    // inputs 3q .. 3q + 2 of group g0 + c, standardised and rounded to bf16 (every lane derives all 12 and
    // keeps its three: no divergence between the lanes of a group)
    bh_bf16x4 x = {0, 0, 0, 0};
    if (c < cnt) {
        const int64_t g = g0 + c;
        const LeafInfo L = leaves[g >> 3];
        float fv[BH_MLP_INPUTS];
        group_features12(n, L, (int)(g >> 3), (int)(g & 7), fv);
        const int f = 3 * q;
        const float a0 = q == 0 ? fv[0] : (q == 1 ? fv[3] : (q == 2 ? fv[6] : fv[9]));
        const float a1 = q == 0 ? fv[1] : (q == 1 ? fv[4] : (q == 2 ? fv[7] : fv[10]));
        const float a2 = q == 0 ? fv[2] : (q == 1 ? fv[5] : (q == 2 ? fv[8] : fv[11]));
        x[0] = bf16_bits((a0 - n.mean[f]) * n.scale[f]);
        x[1] = bf16_bits((a1 - n.mean[f + 1]) * n.scale[f + 1]);
        x[2] = bf16_bits((a2 - n.mean[f + 2]) * n.scale[f + 2]);
    }
    const short *w = reinterpret_cast<const short *>(n.w);
    // layer 1
    bh_bf16x4 h1[4];
#pragma unroll
    for (int t = 0; t < 4; t++) {
        const short *r = w + OW1 + (16 * t + c) * BH_MLP_INPUTS + 3 * q;
        const bh_bf16x4 a = {r[0], r[1], r[2], 0};
        bh_f32x4 acc;
#pragma unroll
        for (int i = 0; i < 4; i++) acc[i] = bf16_load(n.w, OB1 + 16 * t + 4 * q + i);
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, x, acc, 0, 0, 0);
#pragma unroll
        for (int i = 0; i < 4; i++) h1[t][i] = bf16_bits(tanhf(acc[i]));
    }
    // layer 2 and the output's partial sum
    float part = 0.0f;
#pragma unroll
    for (int t = 0; t < 4; t++) {
        bh_f32x4 acc;
#pragma unroll
        for (int i = 0; i < 4; i++) acc[i] = bf16_load(n.w, OB2 + 16 * t + 4 * q + i);
#pragma unroll
        for (int k = 0; k < 4; k++) {
            // W2[16t + c][16k + 4q .. 16k + 4q + 3]: 8 bytes, 8-byte aligned
            const bh_bf16x4 a = *reinterpret_cast<const bh_bf16x4 *>(w + OW2 + (16 * t + c) * BH_MLP_HIDDEN + 16 * k +
                                                                     4 * q);
            acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, h1[k], acc, 0, 0, 0);
        }
#pragma unroll
        for (int i = 0; i < 4; i++) part = fmaf(bf16_load(n.w, OW3 + 16 * t + 4 * q + i), bf16_round(tanhf(acc[i])), part);
    }
    part += __shfl_xor(part, 16, 64);
    part += __shfl_xor(part, 32, 64);
    const float z = part + bf16_load(n.w, OB3);
    const float th = 0.2f + 0.8f / (1.0f + expf(-z)) - n.shift;
    // snapped up to the grid 0.20, 0.25, ..., 1.00 on which the labels and the
    // safety shift are defined (the shift is calibrated charging each
    // prediction the error of the next grid value up): the walk then uses a
    // value whose error was measured, and a network saturating just below 1
    // walks at 1; the network's floor keeps a group off thetas below what it
    // was trained on
    int kk = (int)ceilf((th - 1e-6f - 0.2f) * 20.0f);
    kk = kk < n.kmin ? n.kmin : (kk > 16 ? 16 : kk);
    return (float)(0.2 + 0.05 * (double)kk);
}

}  // namespace bh
