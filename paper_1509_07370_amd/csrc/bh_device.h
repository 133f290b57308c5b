// Small device helpers shared by the kernel sources.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace bh {

// LDS written by one wavefront and read back by the same wavefront: DS
// instructions of a wave execute in order, so only the compiler must be kept
// from moving accesses across this point.
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ int lane_prefix(uint64_t mask) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

__device__ __forceinline__ int morton9(int i, int j, int k) {
    int m = 0;
#pragma unroll
    for (int p = 0; p < 3; p++)
        m |= (((i >> p) & 1) << (3 * p)) | (((j >> p) & 1) << (3 * p + 1)) | (((k >> p) & 1) << (3 * p + 2));
    return m;
}

__device__ __forceinline__ void demorton9(int m, int &i, int &j, int &k) {
    i = j = k = 0;
#pragma unroll
    for (int p = 0; p < 3; p++) {
        i |= ((m >> (3 * p)) & 1) << p;
        j |= ((m >> (3 * p + 1)) & 1) << p;
        k |= ((m >> (3 * p + 2)) & 1) << p;
    }
}

}  // namespace bh
