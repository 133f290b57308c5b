// Periodic Green's function table (device side).
//
// For a cubic box of side L repeated in every direction, the potential of a
// unit mass with the mean density removed is psi(r) = 1/|r| + D(r), D smooth
// in the nearest-image cube (appendix "Periodic boundaries": Ewald's split
// into short- and long-range sums).  D is even in every coordinate, so the
// table covers the octant [0, L/2]^3 on n^3 points with spacing
// sp = (L/2) / (n - 1).  Each point holds D and its derivatives to third
// order (20 values: D; D_x D_y D_z; D_xx D_yy D_zz D_xy D_xz D_yz; D_xxx D_yyy
// D_zzz D_xxy D_xxz D_xyy D_yyz D_xzz D_yzz D_xyz), and a lookup is the
// third-order Taylor expansion about the nearest point (the Hessian: first
// order).  Derivatives of odd order in a coordinate change sign with it.
// The table of 20 values per point is 16-byte aligned per point (80 B in
// fp32, 160 B in fp64).
#pragma once

#include <hip/hip_runtime.h>

#include "bh_internal.h"

namespace bh {

// The compact rows (row (k n + j) n + i for the point (i, j, k) sp) of the
// dimensionless values D L, g L^2, H L^3, T L^4: fp64 walks read 4 fp64 +
// 16 fp32 per point, fp32 walks 4 fp32 + 16 fp16.  Offsets are taken in
// units of L and a lookup gives D L and H L^3 (the caller scales).
template <typename real>
struct EwaldView {
    const real *tab;
    real inv_sp, sp;
    int n;
    real inv_box, sp_box;  // 1 / L and sp / L
};

template <typename real>
struct EwaldPoint {
    uint32_t row;     // table point, (k n + j) n + i
    real dx, dy, dz;  // offset from the table point, folded coordinates
    real sx, sy, sz;  // signs of the coordinates
};

// Nearest table point of R (|R_a| <= L/2 up to rounding; beyond, the last
// point is used and the expansion extrapolates).  Row indices stay below
// 2^31 / 80 for the largest table (129^3 points).
template <typename real>
__device__ __forceinline__ EwaldPoint<real> ewald_point(const EwaldView<real> &e, real rx, real ry, real rz) {
    EwaldPoint<real> p;
    const real ax = fabs(rx), ay = fabs(ry), az = fabs(rz);
    int ix = (int)rint(ax * e.inv_sp), iy = (int)rint(ay * e.inv_sp), iz = (int)rint(az * e.inv_sp);
    ix = ix < e.n - 1 ? ix : e.n - 1;
    iy = iy < e.n - 1 ? iy : e.n - 1;
    iz = iz < e.n - 1 ? iz : e.n - 1;
    p.row = (uint32_t)((iz * e.n + iy) * e.n + ix);
    p.dx = ax * e.inv_box - (real)ix * e.sp_box;
    p.dy = ay * e.inv_box - (real)iy * e.sp_box;
    p.dz = az * e.inv_box - (real)iz * e.sp_box;
    p.sx = copysign((real)1, rx);
    p.sy = copysign((real)1, ry);
    p.sz = copysign((real)1, rz);
    return p;
}

// The 20 values of a table point, as 16-byte loads (issued where called: a
// caller may fetch the next pair's row before it evaluates the current one):
// three for an fp32 row, six for an fp64 row.
typedef _Float16 bh_half8 __attribute__((ext_vector_type(8)));
template <typename real>
__device__ __forceinline__ void ewald_fetch(const EwaldView<real> &e, uint32_t row, real (&v)[kEwaldValues]) {
    if constexpr (sizeof(real) == 4) {
        const float4 *r = reinterpret_cast<const float4 *>(e.tab) + row * 3u;
        const float4 t = r[0];
        const bh_half8 a = *reinterpret_cast<const bh_half8 *>(r + 1);
        const bh_half8 b = *reinterpret_cast<const bh_half8 *>(r + 2);
        v[0] = t.x;
        v[1] = t.y;
        v[2] = t.z;
        v[3] = t.w;
#pragma unroll
        for (int q = 0; q < 8; q++) {
            v[4 + q] = (float)a[q];
            v[12 + q] = (float)b[q];
        }
    } else {
        const double2 *r = reinterpret_cast<const double2 *>(e.tab) + row * 6u;
        const double2 t0 = r[0], t1 = r[1];
        v[0] = t0.x;
        v[1] = t0.y;
        v[2] = t1.x;
        v[3] = t1.y;
        const float4 *f = reinterpret_cast<const float4 *>(r + 2);
#pragma unroll
        for (int q = 0; q < 4; q++) {
            const float4 t = f[q];
            v[4 + 4 * q] = t.x;
            v[5 + 4 * q] = t.y;
            v[6 + 4 * q] = t.z;
            v[7 + 4 * q] = t.w;
        }
    }
}

// D at the point's position (third-order Taylor expansion) and, if H is not
// null, its Hessian (first order; xx yy zz xy xz yz in the caller's
// coordinates), in the table's units: D L and H L^3.  With K = T delta (the third derivatives contracted with the
// offset), the Hessian at the position is H + K and
//   D = D0 + delta . (g + (H + K / 3) delta / 2),
// which is the expansion D0 + g.delta + delta^T H delta / 2 + T[delta^3] / 6.
template <typename real>
__device__ __forceinline__ real ewald_eval(const EwaldPoint<real> &p, const real (&v)[kEwaldValues], real *H) {
    const real x = p.dx, y = p.dy, z = p.dz;
    const real kxx = v[10] * x + v[13] * y + v[14] * z;
    const real kyy = v[15] * x + v[11] * y + v[16] * z;
    const real kzz = v[17] * x + v[18] * y + v[12] * z;
    const real kxy = v[13] * x + v[15] * y + v[19] * z;
    const real kxz = v[14] * x + v[19] * y + v[17] * z;
    const real kyz = v[19] * x + v[16] * y + v[18] * z;
    const real c3 = (real)1 / (real)3, h = (real)0.5;
    const real axx = v[4] + kxx * c3, ayy = v[5] + kyy * c3, azz = v[6] + kzz * c3;
    const real axy = v[7] + kxy * c3, axz = v[8] + kxz * c3, ayz = v[9] + kyz * c3;
    const real wx = axx * x + axy * y + axz * z;
    const real wy = axy * x + ayy * y + ayz * z;
    const real wz = axz * x + ayz * y + azz * z;
    if (H) {
        H[0] = v[4] + kxx;
        H[1] = v[5] + kyy;
        H[2] = v[6] + kzz;
        H[3] = (v[7] + kxy) * (p.sx * p.sy);
        H[4] = (v[8] + kxz) * (p.sx * p.sz);
        H[5] = (v[9] + kyz) * (p.sy * p.sz);
    }
    return v[0] + x * (v[1] + h * wx) + y * (v[2] + h * wy) + z * (v[3] + h * wz);
}

// D at R in one call (point, fetch, evaluate, D L scaled back).
template <typename real>
__device__ __forceinline__ real ewald_value_at(const EwaldView<real> &e, real rx, real ry, real rz) {
    const EwaldPoint<real> p = ewald_point(e, rx, ry, rz);
    real v[kEwaldValues];
    ewald_fetch(e, p.row, v);
    return ewald_eval<real>(p, v, nullptr) * e.inv_box;
}

}  // namespace bh
