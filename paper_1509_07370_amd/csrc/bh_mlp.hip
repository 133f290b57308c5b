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
#include "bh_theta_net.h"

namespace bh {


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


// bf16 copy of the parameters
__global__ void to_bf16_kernel(const float *__restrict__ p, uint16_t *__restrict__ q, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) q[i] = (uint16_t)(__float_as_uint(bf16_round(p[i])) >> 16);
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

// Features and bf16 network in one pass (bh_theta_net.h), 16 groups per
// single-wavefront workgroup; the weights are read from global memory (10 KB,
// cached).
__global__ __launch_bounds__(64) void theta_infer_kernel(const LeafInfo *__restrict__ leaves, int64_t n_groups,
                                                         ThetaNetArgs net, float *__restrict__ theta) {
    const int lane = threadIdx.x;
    const int64_t g0 = (int64_t)blockIdx.x * 16;
    const int cnt = (int)(n_groups - g0 < 16 ? n_groups - g0 : 16);
    const float th = groups_theta16(net, leaves, g0, cnt, lane);
    if (lane < cnt) {
        const int64_t g = g0 + lane;
        theta[(int64_t)leaves[g >> 3].canon * 8 + (g & 7)] = th;
    }
}

ThetaNetArgs theta_net_args(const bh_grid *g, const bh_moments *m, const bh_mlp *net, float shift) {
    ThetaNetArgs a;
    a.w = net->d_bf16;
    a.mean = net->d_mean;
    a.scale = net->d_scale;
    a.shift = shift;
    a.kmin = net->theta_floor_k;
    a.mom = m->d_mom;
    a.geom = g->d_geom;
    a.leaf_parent = g->d_leaf_parent;
    a.root = g->topo.root;
    a.nbase = g->topo.nbase;
    a.box = g->topo.box;
    return a;
}

hipError_t launch_theta_infer(const bh_grid *g, const bh_moments *m, const bh_mlp *net, float shift, float *theta,
                              hipStream_t s) {
    if (g->n_groups == 0) return hipSuccess;
    const int64_t blocks = (g->n_groups + 15) / 16;
    hipLaunchKernelGGL(theta_infer_kernel, dim3((unsigned)blocks), dim3(64), 0, s, g->d_leaves, g->n_groups,
                       theta_net_args(g, m, net, shift), theta);
    return hipGetLastError();
}

hipError_t launch_mlp_bf16(bh_mlp *net, hipStream_t s) {
    hipLaunchKernelGGL(to_bf16_kernel, dim3((kMlpParams + 255) / 256), dim3(256), 0, s, net->d_params, net->d_bf16,
                       kMlpParams);
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
