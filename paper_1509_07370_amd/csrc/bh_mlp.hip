// Learned per-group opening angle: group features, per-group error of a
// potential against a reference, and a 12 -> 64 -> 64 -> 1 MLP (tanh hidden
// units, theta = 0.2 + 0.8 sigmoid(z)) with training (fp32) and bf16 inference.
//
// Parameter vector layout (fp32, kMlpParams = 5057 entries):
//   W1[64][12] | b1[64] | W2[64][64] | b2[64] | W3[64] | b3
// Inputs are normalised as (x - mean) * scale before the first layer.
#include <hip/hip_runtime.h>

#include "bh_device.h"
#include "bh_internal.h"
#include "bh_mlp.h"

namespace bh {

__device__ __forceinline__ float wave_sum(float v) {
    // fixed butterfly order: deterministic
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ double log_floor(double x, double floor) { return log(x > floor ? x : floor); }

// ---------------------------------------------------------------- features

// One thread per group.  Features (per canonical group, 12 floats):
//  0 log2(group cells)                  1 log(M_group / M_root)
//  2 log(group edge / box)              3 AMR level of the leaf block
//  4 log(max / mean cell mass in group) 5,6 log(delta/l), log(|Q|_F/(M l^2)) of the group node
//  7,8 the same for the leaf block      9,10 the same for the block's parent node
// 11 log(mean group density / mean density of its leaf block)
__global__ __launch_bounds__(256) void features_kernel(const LeafInfo *__restrict__ leaves,
                                                       const double *__restrict__ mom,
                                                       const double *__restrict__ geom,
                                                       const int32_t *__restrict__ parent,
                                                       const double4 *__restrict__ cells, int64_t n_groups, int root,
                                                       double box, int nbase, float *__restrict__ out) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= n_groups) return;
    const int f = (int)(g >> 3), sub = (int)(g & 7);
    const LeafInfo L = leaves[f];
    const int node[3] = {L.oct_first + sub, L.block_node, parent[L.block_node] >= 0 ? parent[L.block_node]
                                                                                    : L.block_node};
    const double Mroot = mom[(int64_t)root * kMom + 3];
    const double Mg = mom[(int64_t)node[0] * kMom + 3];
    const double Mb = mom[(int64_t)node[1] * kMom + 3];
    float ft[12];
    ft[0] = 6.0f;
    ft[1] = (float)log_floor(Mroot > 0.0 ? Mg / Mroot : 0.0, 1e-30);
    ft[2] = (float)log(4.0 * L.h / box);
    ft[3] = (float)rint(log2(box / ((double)nbase * kNB * L.h)));
    double mmax = 0.0, msum = 0.0;
    for (int q = 0; q < 64; q++) {
        double m = cells[(int64_t)f * kCellsPerBlock + sub * 64 + q].w;
        msum += m;
        mmax = m > mmax ? m : mmax;
    }
    ft[4] = (float)(msum > 0.0 ? log(mmax / (msum / 64.0)) : 0.0);
    for (int a = 0; a < 3; a++) {
        const double *r = mom + (int64_t)node[a] * kMom;
        const double l = geom[4 * (int64_t)node[a] + 3];
        const double M = r[3];
        const double qf = sqrt(r[4] * r[4] + r[5] * r[5] + r[6] * r[6] + 2.0 * (r[7] * r[7] + r[8] * r[8] + r[9] * r[9]));
        ft[5 + 2 * a] = (float)log(r[10] / l + 1e-6);
        ft[6 + 2 * a] = (float)log((M > 0.0 ? qf / (M * l * l) : 0.0) + 1e-6);
    }
    ft[11] = (float)(Mb > 0.0 ? log_floor(8.0 * Mg / Mb, 1e-30) : 0.0);
    float *o = out + ((int64_t)L.canon * 8 + sub) * kMlpIn;
    for (int k = 0; k < kMlpIn; k++) o[k] = ft[k];
}

hipError_t launch_features(const bh_grid *g, const bh_moments *m, float *out, hipStream_t s) {
    const int blocks = (int)((g->n_groups + 255) / 256);
    hipLaunchKernelGGL(features_kernel, dim3(blocks), dim3(256), 0, s, g->d_leaves, m->d_mom, g->d_geom, g->d_parent,
                       m->d_cell64, g->n_groups, g->topo.root, g->topo.box, g->topo.nbase, out);
    return hipGetLastError();
}

// ---------------------------------------------------------------- per-group error

// One wavefront per group: rms = sqrt(mean_i ((phi_i - ref_i) / ref_i)^2).
__global__ __launch_bounds__(256) void group_rms_kernel(const LeafInfo *__restrict__ leaves, int64_t n_groups,
                                                        const double *__restrict__ phi,
                                                        const double *__restrict__ ref, float *__restrict__ out) {
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t g = (int64_t)blockIdx.x * 4 + w;
    if (g >= n_groups) return;
    const int f = (int)(g >> 3), sub = (int)(g & 7);
    const LeafInfo L = leaves[f];
    int i, j, k;
    demorton9(sub * 64 + lane, i, j, k);
    const int64_t idx = (int64_t)L.canon * kCellsPerBlock + k * 64 + j * 8 + i;
    const double r = (phi[idx] - ref[idx]) / ref[idx];
    const float s = wave_sum((float)(r * r));
    if (lane == 0) out[(int64_t)L.canon * 8 + sub] = sqrtf(s / 64.0f);
}

hipError_t launch_group_rms(const bh_grid *g, const double *phi, const double *ref, float *out, hipStream_t s) {
    const int blocks = (int)((g->n_groups + 3) / 4);
    hipLaunchKernelGGL(group_rms_kernel, dim3(blocks), dim3(256), 0, s, g->d_leaves, g->n_groups, phi, ref, out);
    return hipGetLastError();
}

// ---------------------------------------------------------------- MLP

constexpr int OW1 = 0, OB1 = 768, OW2 = 832, OB2 = 4928, OW3 = 4992, OB3 = 5056;

__device__ __forceinline__ float bf16_round(float x) {
    uint32_t u = __float_as_uint(x);
    u = (u + 0x7FFFu + ((u >> 16) & 1u)) & 0xFFFF0000u;  // round to nearest even
    return __uint_as_float(u);
}
__device__ __forceinline__ float bf16_load(const uint16_t *p, int i) { return __uint_as_float((uint32_t)p[i] << 16); }

// bf16 copy of the parameters, plus W2 transposed for the inference kernel
__global__ void to_bf16_kernel(const float *__restrict__ p, uint16_t *__restrict__ q, uint16_t *__restrict__ w2t,
                               int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint16_t b = (uint16_t)(__float_as_uint(bf16_round(p[i])) >> 16);
    q[i] = b;
    const int r = i - OW2;
    if (r >= 0 && r < kMlpHidden * kMlpHidden) w2t[(r % kMlpHidden) * kMlpHidden + r / kMlpHidden] = b;
}

// One wavefront per sample, lane j = hidden unit j.  BF16: weights, inputs and
// hidden activations rounded to bf16, products accumulated in fp32.
template <bool BF16>
__global__ __launch_bounds__(256) void mlp_forward_kernel(const float *__restrict__ P, const uint16_t *__restrict__ Pb,
                                                          const float *__restrict__ mean,
                                                          const float *__restrict__ scale,
                                                          const float *__restrict__ feat, int64_t n, float shift,
                                                          float *__restrict__ theta) {
    __shared__ float hb[4][64];
    const int w = threadIdx.x >> 6, j = threadIdx.x & 63;
    const int64_t s = (int64_t)blockIdx.x * 4 + w;
    if (s >= n) return;
    float x[kMlpIn];
    for (int i = 0; i < kMlpIn; i++) {
        x[i] = (feat[s * kMlpIn + i] - mean[i]) * scale[i];
        if (BF16) x[i] = bf16_round(x[i]);
    }
    auto W = [&](int i) { return BF16 ? bf16_load(Pb, i) : P[i]; };
    float a = W(OB1 + j);
    for (int i = 0; i < kMlpIn; i++) a = fmaf(W(OW1 + j * kMlpIn + i), x[i], a);
    float h1 = tanhf(a);
    if (BF16) h1 = bf16_round(h1);
    hb[w][j] = h1;
    wave_lds_sync();
    float a2 = W(OB2 + j);
    for (int k = 0; k < kMlpHidden; k++) a2 = fmaf(W(OW2 + j * kMlpHidden + k), hb[w][k], a2);
    float h2 = tanhf(a2);
    if (BF16) h2 = bf16_round(h2);
    const float z = wave_sum(W(OW3 + j) * h2) + W(OB3);
    if (j == 0) {
        const float th = 0.2f + 0.8f / (1.0f + expf(-z)) - shift;
        theta[s] = th < 0.05f ? 0.05f : (th > 1.0f ? 1.0f : th);
    }
}

// Gradient of L = (1/n) sum_s (theta_s - y_s)^2 over a contiguous chunk of
// samples per wavefront, written as one partial gradient per chunk (summed
// later in chunk order, so the result does not depend on scheduling).
__global__ __launch_bounds__(64) void mlp_grad_partial_kernel(const float *__restrict__ P,
                                                              const float *__restrict__ mean,
                                                              const float *__restrict__ scale,
                                                              const float *__restrict__ feat,
                                                              const float *__restrict__ label, int64_t n, int nchunks,
                                                              float *__restrict__ partials) {
    __shared__ float h1s[64];
    __shared__ float d2s[64];
    const int c = blockIdx.x, j = threadIdx.x;
    const int64_t s0 = n * c / nchunks, s1 = n * (c + 1) / nchunks;
    float gW1[kMlpIn], gW2[kMlpHidden];
    for (int i = 0; i < kMlpIn; i++) gW1[i] = 0.f;
    for (int k = 0; k < kMlpHidden; k++) gW2[k] = 0.f;
    float gb1 = 0.f, gb2 = 0.f, gW3 = 0.f, gb3 = 0.f, loss = 0.f;
    const float invn = 1.0f / (float)n;
    for (int64_t s = s0; s < s1; s++) {
        float x[kMlpIn];
        for (int i = 0; i < kMlpIn; i++) x[i] = (feat[s * kMlpIn + i] - mean[i]) * scale[i];
        float a = P[OB1 + j];
        for (int i = 0; i < kMlpIn; i++) a = fmaf(P[OW1 + j * kMlpIn + i], x[i], a);
        const float h1 = tanhf(a);
        h1s[j] = h1;
        __syncthreads();
        float a2 = P[OB2 + j];
        for (int k = 0; k < kMlpHidden; k++) a2 = fmaf(P[OW2 + j * kMlpHidden + k], h1s[k], a2);
        const float h2 = tanhf(a2);
        const float z = wave_sum(P[OW3 + j] * h2) + P[OB3];
        const float sg = 1.0f / (1.0f + expf(-z));
        const float th = 0.2f + 0.8f * sg;
        const float e = th - label[s];
        loss += e * e * invn;
        const float dz = 2.0f * e * invn * 0.8f * sg * (1.0f - sg);
        gb3 += dz;
        gW3 = fmaf(dz, h2, gW3);
        const float d2 = dz * P[OW3 + j] * (1.0f - h2 * h2);
        gb2 += d2;
        for (int k = 0; k < kMlpHidden; k++) gW2[k] = fmaf(d2, h1s[k], gW2[k]);
        d2s[j] = d2;
        __syncthreads();
        float d1 = 0.f;  // lane j = input unit k = j of layer 2
        for (int q = 0; q < kMlpHidden; q++) d1 = fmaf(P[OW2 + q * kMlpHidden + j], d2s[q], d1);
        d1 *= (1.0f - h1 * h1);
        gb1 += d1;
        for (int i = 0; i < kMlpIn; i++) gW1[i] = fmaf(d1, x[i], gW1[i]);
        __syncthreads();
    }
    float *o = partials + (int64_t)c * (kMlpParams + 1);
    for (int i = 0; i < kMlpIn; i++) o[OW1 + j * kMlpIn + i] = gW1[i];
    o[OB1 + j] = gb1;
    for (int k = 0; k < kMlpHidden; k++) o[OW2 + j * kMlpHidden + k] = gW2[k];
    o[OB2 + j] = gb2;
    o[OW3 + j] = gW3;
    if (j == 0) {
        o[OB3] = gb3;
        o[kMlpParams] = loss;
    }
}

__global__ __launch_bounds__(256) void mlp_grad_reduce_kernel(const float *__restrict__ partials, int nchunks,
                                                              float *__restrict__ grad, float *__restrict__ loss) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p > kMlpParams) return;
    float acc = 0.f;
    for (int c = 0; c < nchunks; c++) acc += partials[(int64_t)c * (kMlpParams + 1) + p];
    if (p < kMlpParams)
        grad[p] = acc;
    else if (loss)
        *loss = acc;
}

__global__ __launch_bounds__(256) void mlp_adam_kernel(float *__restrict__ P, float *__restrict__ M,
                                                       float *__restrict__ V, const float *__restrict__ grad, float lr,
                                                       float b1, float b2, float eps, float c1, float c2) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= kMlpParams) return;
    const float g = grad[p];
    const float m = b1 * M[p] + (1.0f - b1) * g;
    const float v = b2 * V[p] + (1.0f - b2) * g * g;
    M[p] = m;
    V[p] = v;
    P[p] -= lr * (m / c1) / (sqrtf(v / c2) + eps);
}

// Features and bf16 network in one pass, four lanes per group (64 groups per
// 256-thread workgroup).  The features come from node rows only (the largest
// cell mass of the group's node is kept by the moments kernel in slot 11 of
// its row): lane 0 of a group derives the group-level features, lanes 1..3
// those of the three ancestor nodes.  Each lane then evaluates 16 hidden
// units of both layers (16 independent accumulators) with the bf16 weights
// staged once per workgroup in LDS -- W2 transposed, so that a lane reads its
// 16 weights of one input in two 16-byte loads -- and the four partial output
// sums of a group are added across its lanes.
constexpr int kInferGroups = 64;   // groups per workgroup
constexpr int kInferUnits = 16;    // hidden units per lane

__device__ __forceinline__ void bf16x8_to_f32(const uint4 v, float *o) {
    const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int i = 0; i < 4; i++) {
        o[2 * i] = __uint_as_float(w[i] << 16);
        o[2 * i + 1] = __uint_as_float(w[i] & 0xFFFF0000u);
    }
}

__global__ __launch_bounds__(256) void theta_infer_kernel(const LeafInfo *__restrict__ leaves,
                                                          const double *__restrict__ mom,
                                                          const double *__restrict__ geom,
                                                          const int32_t *__restrict__ parent, int64_t n_groups,
                                                          int root, double box, int nbase,
                                                          const uint16_t *__restrict__ Pb,
                                                          const uint4 *__restrict__ W2t,
                                                          const float *__restrict__ mean,
                                                          const float *__restrict__ scale, float shift,
                                                          float *__restrict__ theta) {
    __shared__ __align__(16) uint16_t w2t[kMlpHidden * kMlpHidden];  // [k][u] = W2[u][k]
    __shared__ uint16_t w1[kMlpHidden * kMlpIn + kMlpHidden];        // W1 then b1
    __shared__ uint16_t w23[2 * kMlpHidden + 1];                     // b2, w3, b3
    __shared__ float xs[kInferGroups][kMlpIn + 1];
    __shared__ float h1s[kInferGroups][kMlpHidden + 1];
    for (int i = threadIdx.x; i < kMlpHidden * kMlpHidden / 8; i += blockDim.x)
        reinterpret_cast<uint4 *>(w2t)[i] = W2t[i];
    for (int i = threadIdx.x; i < kMlpHidden * kMlpIn + kMlpHidden; i += blockDim.x) w1[i] = Pb[OW1 + i];
    for (int i = threadIdx.x; i < 2 * kMlpHidden + 1; i += blockDim.x) w23[i] = Pb[OB2 + i];
    const int gl = threadIdx.x >> 2, q = threadIdx.x & 3;
    const int64_t g = (int64_t)blockIdx.x * kInferGroups + gl;
    const bool valid = g < n_groups;
    LeafInfo L{};
    int sub = 0;
    if (valid) {
        const int f = (int)(g >> 3);
        sub = (int)(g & 7);
        L = leaves[f];
        const int gnode = L.oct_first + sub;
        const double Mg = mom[(int64_t)gnode * kMom + 3];
        float ft[3];
        int nft, first;
        if (q == 0) {
            const double Mroot = mom[(int64_t)root * kMom + 3];
            const double Mb = mom[(int64_t)L.block_node * kMom + 3];
            const double mmax = mom[(int64_t)gnode * kMom + 11];
            xs[gl][0] = 6.0f;
            xs[gl][1] = (float)log_floor(Mroot > 0.0 ? Mg / Mroot : 0.0, 1e-30);
            xs[gl][2] = (float)log(4.0 * L.h / box);
            xs[gl][3] = (float)rint(log2(box / ((double)nbase * kNB * L.h)));
            xs[gl][4] = (float)(Mg > 0.0 ? log(mmax / (Mg / 64.0)) : 0.0);
            ft[0] = (float)(Mb > 0.0 ? log_floor(8.0 * Mg / Mb, 1e-30) : 0.0);
            nft = 1;
            first = 11;
        } else {
            const int a = q - 1;
            const int pn = parent[L.block_node];
            const int node = a == 0 ? gnode : (a == 1 ? L.block_node : (pn >= 0 ? pn : L.block_node));
            const double *r = mom + (int64_t)node * kMom;
            const double l = geom[4 * (int64_t)node + 3];
            const double M = r[3];
            const double qf = sqrt(r[4] * r[4] + r[5] * r[5] + r[6] * r[6] +
                                   2.0 * (r[7] * r[7] + r[8] * r[8] + r[9] * r[9]));
            ft[0] = (float)log(r[10] / l + 1e-6);
            ft[1] = (float)log((M > 0.0 ? qf / (M * l * l) : 0.0) + 1e-6);
            nft = 2;
            first = 5 + 2 * a;
        }
        for (int i = 0; i < nft; i++) xs[gl][first + i] = ft[i];
    }
    __syncthreads();
    if (valid && q == 0)
        for (int i = 0; i < kMlpIn; i++) xs[gl][i] = bf16_round((xs[gl][i] - mean[i]) * scale[i]);
    __syncthreads();
    const int u0 = q * kInferUnits;
    if (valid) {
        float x[kMlpIn];
        for (int i = 0; i < kMlpIn; i++) x[i] = xs[gl][i];
        for (int j = 0; j < kInferUnits; j++) {
            const int u = u0 + j;
            float a1 = bf16_load(w1, kMlpHidden * kMlpIn + u);
            for (int i = 0; i < kMlpIn; i++) a1 = fmaf(bf16_load(w1, u * kMlpIn + i), x[i], a1);
            h1s[gl][u] = bf16_round(tanhf(a1));
        }
    }
    __syncthreads();
    if (!valid) return;
    float acc[kInferUnits];
    for (int j = 0; j < kInferUnits; j++) acc[j] = bf16_load(w23, u0 + j);
    for (int k = 0; k < kMlpHidden; k++) {
        const float hk = h1s[gl][k];
        const uint4 *row = reinterpret_cast<const uint4 *>(w2t + k * kMlpHidden + u0);
        float w[kInferUnits];
        bf16x8_to_f32(row[0], w);
        bf16x8_to_f32(row[1], w + 8);
#pragma unroll
        for (int j = 0; j < kInferUnits; j++) acc[j] = fmaf(w[j], hk, acc[j]);
    }
    float z = 0.0f;
    for (int j = 0; j < kInferUnits; j++) z = fmaf(bf16_load(w23, kMlpHidden + u0 + j), bf16_round(tanhf(acc[j])), z);
    z += __shfl_xor(z, 1, 64);
    z += __shfl_xor(z, 2, 64);
    if (q == 0) {
        z += bf16_load(w23, 2 * kMlpHidden);
        const float th = 0.2f + 0.8f / (1.0f + expf(-z)) - shift;
        theta[(int64_t)L.canon * 8 + sub] = th < 0.05f ? 0.05f : (th > 1.0f ? 1.0f : th);
    }
}

hipError_t launch_theta_infer(const bh_grid *g, const bh_moments *m, const bh_mlp *net, float shift, float *theta,
                              hipStream_t s) {
    const int blocks = (int)((g->n_groups + kInferGroups - 1) / kInferGroups);
    hipLaunchKernelGGL(theta_infer_kernel, dim3(blocks), dim3(256), 0, s, g->d_leaves, m->d_mom, g->d_geom,
                       g->d_parent, g->n_groups, g->topo.root, g->topo.box, g->topo.nbase, net->d_bf16,
                       reinterpret_cast<const uint4 *>(net->d_w2t), net->d_mean, net->d_scale, shift, theta);
    return hipGetLastError();
}

hipError_t launch_mlp_bf16(bh_mlp *net, hipStream_t s) {
    hipLaunchKernelGGL(to_bf16_kernel, dim3((kMlpParams + 255) / 256), dim3(256), 0, s, net->d_params, net->d_bf16,
                       net->d_w2t, kMlpParams);
    return hipGetLastError();
}

hipError_t launch_mlp_forward(const bh_mlp *net, const float *feat, int64_t n, bool bf16, float shift, float *theta,
                              hipStream_t s) {
    if (n == 0) return hipSuccess;
    const int blocks = (int)((n + 3) / 4);
    if (bf16)
        hipLaunchKernelGGL(mlp_forward_kernel<true>, dim3(blocks), dim3(256), 0, s, net->d_params, net->d_bf16,
                           net->d_mean, net->d_scale, feat, n, shift, theta);
    else
        hipLaunchKernelGGL(mlp_forward_kernel<false>, dim3(blocks), dim3(256), 0, s, net->d_params, net->d_bf16,
                           net->d_mean, net->d_scale, feat, n, shift, theta);
    return hipGetLastError();
}

hipError_t launch_mlp_grad(bh_mlp *net, const float *feat, const float *label, int64_t n, float *grad, float *loss,
                           hipStream_t s) {
    const int nchunks = (int)(n < kMlpChunks ? n : kMlpChunks);
    hipLaunchKernelGGL(mlp_grad_partial_kernel, dim3(nchunks), dim3(64), 0, s, net->d_params, net->d_mean,
                       net->d_scale, feat, label, n, nchunks, net->d_partials);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(mlp_grad_reduce_kernel, dim3((kMlpParams + 1 + 255) / 256), dim3(256), 0, s, net->d_partials,
                       nchunks, grad, loss);
    return hipGetLastError();
}

hipError_t launch_mlp_adam(bh_mlp *net, const float *grad, float lr, float b1, float b2, float eps, hipStream_t s) {
    net->step++;
    const float c1 = 1.0f - powf(b1, (float)net->step);
    const float c2 = 1.0f - powf(b2, (float)net->step);
    hipLaunchKernelGGL(mlp_adam_kernel, dim3((kMlpParams + 255) / 256), dim3(256), 0, s, net->d_params, net->d_m,
                       net->d_v, grad, lr, b1, b2, eps, c1, c2);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_mlp_bf16(net, s);
}

}  // namespace bh
