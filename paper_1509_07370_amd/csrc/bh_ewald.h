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
#pragma once

#include <hip/hip_runtime.h>

#include "bh_internal.h"

namespace bh {

template <typename real>
struct EwaldView {
    const real *tab;  // [n][n][n][kEwaldValues], index (k n + j) n + i for u = (i, j, k) sp
    real inv_sp, sp;
    int n;
};

template <typename real>
struct EwaldPoint {
    const real *v;
    real dx, dy, dz;  // offset from the table point, folded coordinates
    real sx, sy, sz;  // signs of the coordinates
};

// Nearest table point of R (|R_a| <= L/2 up to rounding; beyond, the last
// point is used and the expansion extrapolates).
template <typename real>
__device__ __forceinline__ EwaldPoint<real> ewald_point(const EwaldView<real> &e, real rx, real ry, real rz) {
    EwaldPoint<real> p;
    const real ax = rx < (real)0 ? -rx : rx, ay = ry < (real)0 ? -ry : ry, az = rz < (real)0 ? -rz : rz;
    int ix = (int)rint(ax * e.inv_sp), iy = (int)rint(ay * e.inv_sp), iz = (int)rint(az * e.inv_sp);
    ix = ix < e.n - 1 ? ix : e.n - 1;
    iy = iy < e.n - 1 ? iy : e.n - 1;
    iz = iz < e.n - 1 ? iz : e.n - 1;
    p.v = e.tab + ((int64_t)(iz * e.n + iy) * e.n + ix) * kEwaldValues;
    p.dx = ax - (real)ix * e.sp;
    p.dy = ay - (real)iy * e.sp;
    p.dz = az - (real)iz * e.sp;
    p.sx = rx < (real)0 ? (real)-1 : (real)1;
    p.sy = ry < (real)0 ? (real)-1 : (real)1;
    p.sz = rz < (real)0 ? (real)-1 : (real)1;
    return p;
}

// D at the point's position (third-order Taylor expansion).
template <typename real>
__device__ __forceinline__ real ewald_value(const EwaldPoint<real> &p) {
    const real *v = p.v;
    const real x = p.dx, y = p.dy, z = p.dz;
    const real x2 = x * x, y2 = y * y, z2 = z * z;
    const real lin = v[1] * x + v[2] * y + v[3] * z;
    const real quad = (real)0.5 * (v[4] * x2 + v[5] * y2 + v[6] * z2) + (v[7] * x * y + v[8] * x * z + v[9] * y * z);
    const real cub = v[10] * x2 * x + v[11] * y2 * y + v[12] * z2 * z +
                     (real)3 * (v[13] * x2 * y + v[14] * x2 * z + v[15] * x * y2 + v[16] * y2 * z + v[17] * x * z2 +
                                v[18] * y * z2) +
                     (real)6 * v[19] * x * y * z;
    return v[0] + lin + quad + cub * ((real)1 / (real)6);
}

// Hessian of D at the point's position in the caller's coordinates, order
// xx yy zz xy xz yz (first-order expansion, signs unfolded).
template <typename real>
__device__ __forceinline__ void ewald_hessian(const EwaldPoint<real> &p, real *H) {
    const real *v = p.v;
    const real x = p.dx, y = p.dy, z = p.dz;
    H[0] = v[4] + v[10] * x + v[13] * y + v[14] * z;
    H[1] = v[5] + v[15] * x + v[11] * y + v[16] * z;
    H[2] = v[6] + v[17] * x + v[18] * y + v[12] * z;
    H[3] = (v[7] + v[13] * x + v[15] * y + v[19] * z) * (p.sx * p.sy);
    H[4] = (v[8] + v[14] * x + v[19] * y + v[17] * z) * (p.sx * p.sz);
    H[5] = (v[9] + v[19] * x + v[16] * y + v[18] * z) * (p.sy * p.sz);
}

}  // namespace bh
