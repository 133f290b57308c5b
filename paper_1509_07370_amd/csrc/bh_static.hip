// bh_potential_static: the upward pass followed by the fused walk + sums
// (bh_build_moments then bh_walk_potential) with every per-call device
// workspace carved out of one file-scope device array instead of a moments
// handle, so that the call allocates nothing.  It runs the same kernels as
// those two entry points; only where their workspace lives differs.
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>
#include <string>

#include "bh_internal.h"

namespace bh {

// Static scratch: node moments and walk/far records, cell records, per-group
// costs and the status flags of one call.  Each device holds its own copy
// from the moment the library's code object is loaded on it until the
// process ends.
constexpr size_t kStaticScratchBytes = (size_t)BH_STATIC_SCRATCH_BYTES;
constexpr int kMaxStaticDevices = 64;

}  // namespace bh

static __device__ __align__(256) unsigned char scratch[bh::kStaticScratchBytes];

namespace bh {

namespace {

std::mutex g_scratch_lock;
void *g_scratch_ptr[kMaxStaticDevices] = {};

__global__ void clear_ints_kernel(int *p, int n) {
    const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (i < n) p[i] = 0;
}

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

// Byte offsets of each workspace inside the scratch, for one grid.
struct StaticLayout {
    size_t mom, s, brow, w32, w64, f32, cell64, cell32, cost, flags, total;
};

StaticLayout static_layout(const bh_grid *g) {
    const size_t nn = (size_t)g->topo.n_nodes, nc = (size_t)g->n_cells, nl = g->topo.leaves.size();
    const size_t nu = (size_t)g->n_units;
    StaticLayout L{};
    size_t o = 0;
    L.mom = o;
    o = align256(o + nn * kMom * sizeof(double));
    L.s = o;
    o = align256(o + nn * sizeof(double));
    L.brow = o;
    o = align256(o + nl * kBlockRow * sizeof(double));
    L.w32 = o;
    o = align256(o + nn * sizeof(WalkRec32));
    L.w64 = o;
    o = align256(o + nn * sizeof(WalkRec64));
    L.f32 = o;
    o = align256(o + nn * sizeof(FarRec32));
    L.cell64 = o;
    o = align256(o + nc * sizeof(double4));
    L.cell32 = o;
    o = align256(o + nc * sizeof(float4));
    L.cost = o;
    o = align256(o + nu * sizeof(uint32_t));
    L.flags = o;
    o = align256(o + 2 * sizeof(int));
    L.total = o;
    return L;
}

}  // namespace

// Device address of this device's scratch, looked up once per device with
// that device current (the array's name is only a host-side stand-in).
hipError_t static_scratch_setup(int device, void **out) {
    if (device < 0 || device >= kMaxStaticDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_lock);
    if (!g_scratch_ptr[device]) {
        int cur = -1;
        hipError_t e = hipGetDevice(&cur);
        if (e != hipSuccess) return e;
        if (cur != device && (e = hipSetDevice(device)) != hipSuccess) return e;
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur != device) (void)hipSetDevice(cur);
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_ptr[device] = p;
    }
    if (out) *out = g_scratch_ptr[device];
    return hipSuccess;
}

}  // namespace bh

extern "C" int bh_potential_static(bh_ctx *ctx, const bh_grid *g, const double *rho, double theta,
                                   const float *theta_group, int precision, double G, double *phi, int32_t *counts,
                                   int32_t *status) {
    if (!ctx) return BH_EINVAL;
    auto fail = [ctx](int code, const std::string &msg) {
        ctx->err = msg;
        return code;
    };
    auto hip_fail = [&fail](hipError_t e, const char *what) {
        return fail(e == hipErrorOutOfMemory ? BH_ENOMEM : BH_EDEVICE,
                    std::string(what) + ": " + hipGetErrorName(e) + " (" + hipGetErrorString(e) + ")");
    };
    if (ctx->device < 0) return fail(BH_ESTATE, "host-only context: no GPU work possible");
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    if (!g || !rho || !phi) return fail(BH_EINVAL, "grid, rho_dev or phi_dev is NULL");
    if (g->device != ctx->device) return fail(BH_ESTATE, "grid was created on another device");
    if (precision != BH_FP64 && precision != BH_FP32) return fail(BH_EINVAL, "precision must be BH_FP64 or BH_FP32");
    if (!theta_group && !(theta > 0.0 && theta <= 1.0)) return fail(BH_EINVAL, "theta must be in (0, 1]");
    if (!std::isfinite(G)) return fail(BH_EINVAL, "G must be finite");
    const bh::StaticLayout lay = bh::static_layout(g);
    if (lay.total > bh::kStaticScratchBytes)
        return fail(BH_ECAPACITY, "grid needs " + std::to_string(lay.total) + " bytes of workspace; the static scratch holds " +
                                      std::to_string(bh::kStaticScratchBytes));
    void *base = nullptr;
    if ((e = bh::static_scratch_setup(ctx->device, &base)) != hipSuccess) return hip_fail(e, "static scratch address");
    unsigned char *p = (unsigned char *)base;
    // a moments view of the scratch: no schedule (natural dispatch order), fixed epoch 1 on cleared flags
    bh_moments m;
    m.grid = g;
    m.device = ctx->device;
    m.d_mom = (double *)(p + lay.mom);
    m.d_s = (double *)(p + lay.s);
    m.d_brow = (double *)(p + lay.brow);
    m.d_w32 = (bh::WalkRec32 *)(p + lay.w32);
    m.d_w64 = (bh::WalkRec64 *)(p + lay.w64);
    m.d_f32 = (bh::FarRec32 *)(p + lay.f32);
    m.d_cell64 = (double4 *)(p + lay.cell64);
    m.d_cell32 = (float4 *)(p + lay.cell32);
    m.d_cost = (uint32_t *)(p + lay.cost);
    m.d_flags = status ? (int *)status : (int *)(p + lay.flags);
    m.walk_epoch = 1;
    hipLaunchKernelGGL(bh::clear_ints_kernel, dim3(1), dim3(64), 0, ctx->stream, m.d_flags, 2);
    if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "status clear kernel");
    if ((e = bh::launch_moments(g, &m, rho, ctx->stream, 1, false)) != hipSuccess) return hip_fail(e, "moments kernels");
    if ((e = bh::launch_walk_potential(g, &m, theta, theta_group, precision, G, phi, counts, ctx->stream)) != hipSuccess)
        return hip_fail(e, "fused walk + potential kernel");
    return BH_OK;
}
