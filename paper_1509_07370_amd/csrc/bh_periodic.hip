// Periodic boundaries: the Green's function table and the periodic direct
// sum (appendix "Periodic boundaries").
//
//   ewald_table_kernel     one thread per table point: D = psi - 1/|r| and its
//                          derivatives to third order from Ewald's sums (fp64)
//   direct_periodic_kernel exact-method reference: every pair through the
//                          nearest image and the table, fp64
#include <hip/hip_runtime.h>

#include "bh_device.h"
#include "bh_ewald.h"
#include "bh_internal.h"

namespace bh {

// Accumulator of D, its gradient, Hessian (xx yy zz xy xz yz) and third
// derivatives (xxx yyy zzz xxy xxz xyy yyz xzz yzz xyz).
struct EwaldAcc {
    double v[kEwaldValues];
};

// Adds a function of r = |p| given through G1 = f'/r, G2 = G1'/r and
// G3 = G2'/r: gradient G1 p, Hessian G1 I + G2 p p^T, third derivatives
// G2 (I p)_sym + G3 p p p.
__device__ void add_radial_g(EwaldAcc &a, const double *p, double f, double G1, double G2, double G3) {
    const double x = p[0], y = p[1], z = p[2];
    a.v[0] += f;
    a.v[1] += G1 * x;
    a.v[2] += G1 * y;
    a.v[3] += G1 * z;
    a.v[4] += G1 + G2 * x * x;
    a.v[5] += G1 + G2 * y * y;
    a.v[6] += G1 + G2 * z * z;
    a.v[7] += G2 * x * y;
    a.v[8] += G2 * x * z;
    a.v[9] += G2 * y * z;
    a.v[10] += 3.0 * G2 * x + G3 * x * x * x;  // xxx
    a.v[11] += 3.0 * G2 * y + G3 * y * y * y;  // yyy
    a.v[12] += 3.0 * G2 * z + G3 * z * z * z;  // zzz
    a.v[13] += G2 * y + G3 * x * x * y;        // xxy
    a.v[14] += G2 * z + G3 * x * x * z;        // xxz
    a.v[15] += G2 * x + G3 * x * y * y;        // xyy
    a.v[16] += G2 * z + G3 * y * y * z;        // yyz
    a.v[17] += G2 * x + G3 * x * z * z;        // xzz
    a.v[18] += G2 * y + G3 * y * z * z;        // yzz
    a.v[19] += G3 * x * y * z;                 // xyz
}

// The Ewald sums at u for a box of side L, splitting constant a = 2 / L:
//   psi(r) = sum_n erfc(a |r + n L|) / |r + n L|
//          + (1 / (pi L)) sum_{m != 0} exp(-pi^2 |m|^2 / (a L)^2) / |m|^2 cos(2 pi m.r / L)
//          - pi / (a^2 L^3),
// minus 1/|r|.  Images with a |r + n L| > 6.5 (erfc below 1e-19) and wave
// vectors with a component beyond 4 (weights below 1e-17) are left out.
__device__ void ewald_sums(double L, const double *u, EwaldAcc &acc) {
    const double pi = 3.14159265358979323846;
    const double a = 2.0 / L, a2 = a * a;
    const double c = 2.0 * a / 1.7724538509055160273;  // 2 a / sqrt(pi)
    for (int q = 0; q < kEwaldValues; q++) acc.v[q] = 0.0;
    // image 0 less 1/r: -erf(a r)/r, even and smooth
    const double r2 = u[0] * u[0] + u[1] * u[1] + u[2] * u[2], r = sqrt(r2);
    if (a * r < 0.3) {
        // -erf(a r)/r = -c sum_k b_k w^k, w = (a r)^2, b_k = (-1)^k / (k! (2k + 1));
        // G1, G2, G3 from the same series (w^(k-1), w^(k-2), w^(k-3)); to w^11
        // the rest is below 1e-19 for a r < 0.3, where the closed forms below
        // would lose digits to cancellation in G2 and G3
        const double w = a2 * r2;
        double f = 0.0, G1 = 0.0, G2 = 0.0, G3 = 0.0, fact = 1.0;
        for (int k = 0; k <= 11; k++) {
            if (k > 0) fact *= -1.0 / k;
            const double b = fact / (2 * k + 1);
            f += b * pow(w, (double)k);
            if (k >= 1) G1 += b * 2.0 * k * a2 * pow(w, (double)(k - 1));
            if (k >= 2) G2 += b * 2.0 * k * (2.0 * k - 2.0) * a2 * a2 * pow(w, (double)(k - 2));
            if (k >= 3) G3 += b * 2.0 * k * (2.0 * k - 2.0) * (2.0 * k - 4.0) * a2 * a2 * a2 * pow(w, (double)(k - 3));
        }
        add_radial_g(acc, u, -c * f, -c * G1, -c * G2, -c * G3);
    } else {
        const double E = exp(-a2 * r2), ef = erf(a * r);
        const double f = -ef / r;
        const double f1 = ef / r2 - c * E / r;
        const double f2 = 2.0 * c * a2 * E + 2.0 * c * E / r2 - 2.0 * ef / (r2 * r);
        const double f3 = -4.0 * c * a2 * a2 * r * E - 4.0 * c * a2 * E / r - 6.0 * c * E / (r2 * r) + 6.0 * ef / (r2 * r2);
        const double G1 = f1 / r, A = f2 - f1 / r;
        const double G2 = A / r2, G3 = (f3 - 3.0 * f2 / r + 3.0 * f1 / r2) / (r2 * r);
        add_radial_g(acc, u, f, G1, G2, G3);
    }
    for (int i = -3; i <= 3; i++)
        for (int j = -3; j <= 3; j++)
            for (int k = -3; k <= 3; k++) {
                if (i == 0 && j == 0 && k == 0) continue;
                const double p[3] = {u[0] + i * L, u[1] + j * L, u[2] + k * L};
                const double d2 = p[0] * p[0] + p[1] * p[1] + p[2] * p[2], d = sqrt(d2);
                if (a * d > 6.5) continue;
                const double E = exp(-a2 * d2), ec = erfc(a * d);
                const double f1 = -ec / d2 - c * E / d;
                const double f2 = 2.0 * c * a2 * E + 2.0 * c * E / d2 + 2.0 * ec / (d2 * d);
                const double f3 = -4.0 * c * a2 * a2 * d * E - 4.0 * c * a2 * E / d - 6.0 * c * E / (d2 * d) -
                                  6.0 * ec / (d2 * d2);
                add_radial_g(acc, p, ec / d, f1 / d, (f2 - f1 / d) / d2, (f3 - 3.0 * f2 / d + 3.0 * f1 / d2) / (d2 * d));
            }
    // wave vectors: weight and phase factor over the axes
    const double kk = 2.0 * pi / L;
    double ew[9], cs[3][9], sn[3][9];
    for (int m = -4; m <= 4; m++) {
        ew[m + 4] = exp(-pi * pi * (double)(m * m) / (a2 * L * L));
        for (int d = 0; d < 3; d++) sincos(kk * m * u[d], &sn[d][m + 4], &cs[d][m + 4]);
    }
    for (int i = -4; i <= 4; i++)
        for (int j = -4; j <= 4; j++) {
            const double cxy = cs[0][i + 4] * cs[1][j + 4] - sn[0][i + 4] * sn[1][j + 4];
            const double sxy = sn[0][i + 4] * cs[1][j + 4] + cs[0][i + 4] * sn[1][j + 4];
            for (int k = -4; k <= 4; k++) {
                if (i == 0 && j == 0 && k == 0) continue;
                const double m2 = (double)(i * i + j * j + k * k);
                const double w = ew[i + 4] * ew[j + 4] * ew[k + 4] / (pi * L * m2);
                const double co = cxy * cs[2][k + 4] - sxy * sn[2][k + 4];
                const double si = sxy * cs[2][k + 4] + cxy * sn[2][k + 4];
                const double mi = i * kk, mj = j * kk, mk = k * kk;
                // d/du of w cos(m.u k): -w sin (k m); second: -w cos (k m)(k m); third: +w sin (k m)^3
                acc.v[0] += w * co;
                acc.v[1] -= w * si * mi;
                acc.v[2] -= w * si * mj;
                acc.v[3] -= w * si * mk;
                acc.v[4] -= w * co * mi * mi;
                acc.v[5] -= w * co * mj * mj;
                acc.v[6] -= w * co * mk * mk;
                acc.v[7] -= w * co * mi * mj;
                acc.v[8] -= w * co * mi * mk;
                acc.v[9] -= w * co * mj * mk;
                acc.v[10] += w * si * mi * mi * mi;
                acc.v[11] += w * si * mj * mj * mj;
                acc.v[12] += w * si * mk * mk * mk;
                acc.v[13] += w * si * mi * mi * mj;
                acc.v[14] += w * si * mi * mi * mk;
                acc.v[15] += w * si * mi * mj * mj;
                acc.v[16] += w * si * mj * mj * mk;
                acc.v[17] += w * si * mi * mk * mk;
                acc.v[18] += w * si * mj * mk * mk;
                acc.v[19] += w * si * mi * mj * mk;
            }
        }
    acc.v[0] -= pi / (a2 * L * L * L);
}

__global__ __launch_bounds__(128) void ewald_table_kernel(double L, int n, double sp, double *__restrict__ t64,
                                                          double *__restrict__ t64c, float *__restrict__ t32) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t total = (int64_t)n * n * n;
    if (q >= total) return;
    const int i = (int)(q % n), j = (int)((q / n) % n), k = (int)(q / ((int64_t)n * n));
    const double u[3] = {i * sp, j * sp, k * sp};
    EwaldAcc acc;
    ewald_sums(L, u, acc);
    for (int v = 0; v < kEwaldValues; v++) t64[q * kEwaldValues + v] = acc.v[v];
    // compact rows, dimensionless: D L, g L^2, H L^3, T L^4 (magnitudes up to a
    // few hundred, far inside the fp16 range)
    const double L2 = L * L, L3 = L2 * L, L4 = L3 * L;
    double s[kEwaldValues];
    s[0] = acc.v[0] * L;
    for (int v = 1; v < 4; v++) s[v] = acc.v[v] * L2;
    for (int v = 4; v < 10; v++) s[v] = acc.v[v] * L3;
    for (int v = 10; v < kEwaldValues; v++) s[v] = acc.v[v] * L4;
    double *rd = t64c + q * kEwaldCompactDoubles;  // 4 fp64, then 16 fp32
    float *rf = t32 + q * kEwaldCompactFloats;     // 4 fp32, then 16 fp16
    float *rd_hi = reinterpret_cast<float *>(rd + 4);
    _Float16 *rf_hi = reinterpret_cast<_Float16 *>(rf + 4);
    for (int v = 0; v < 4; v++) {
        rd[v] = s[v];
        rf[v] = (float)s[v];
    }
    for (int v = 4; v < kEwaldValues; v++) {
        rd_hi[v - 4] = (float)s[v];
        rf_hi[v - 4] = (_Float16)(float)s[v];
    }
}

// D L (dimensionless) at points u given in units of L, one thread per point:
// the same Ewald sums as the table, at any point (the near-origin series is
// fitted to and checked against these).
__global__ __launch_bounds__(128) void ewald_points_kernel(double L, const double *__restrict__ u, int n,
                                                           double *__restrict__ out) {
    const int q = blockIdx.x * 128 + threadIdx.x;
    if (q >= n) return;
    const double p[3] = {u[3 * q] * L, u[3 * q + 1] * L, u[3 * q + 2] * L};
    EwaldAcc acc;
    ewald_sums(L, p, acc);
    out[q] = acc.v[0] * L;
}

hipError_t launch_ewald_points(double L, const double *u, int n, double *out, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(ewald_points_kernel, dim3((unsigned)((n + 127) / 128)), dim3(128), 0, s, L, u, n, out);
    return hipGetLastError();
}

hipError_t launch_ewald_table(const bh_ewald *e, hipStream_t s) {
    const int64_t total = (int64_t)e->n * e->n * e->n;
    hipLaunchKernelGGL(ewald_table_kernel, dim3((unsigned)((total + 127) / 128)), dim3(128), 0, s, e->L, e->n, e->sp,
                       e->d_t64, e->d_t64c, e->d_t32);
    return hipGetLastError();
}

// Periodic direct sum at selected cells (canonical ids):
//   phi_i = -G [ sum_{j != i} m_j / |R_ij| + sum_j m_j D(R_ij) ],
// R_ij the nearest image of r_i - r_j, D from the table (j = i: D(0), the
// cell's own images).
__global__ __launch_bounds__(256) void direct_periodic_kernel(const int64_t *__restrict__ targets, int64_t n,
                                                              const double4 *__restrict__ cells, int64_t ncells,
                                                              const int32_t *__restrict__ internal_of_canon,
                                                              EwaldView<double> ew, double L, double G,
                                                              double *__restrict__ phi) {
    __shared__ double4 tile[256];
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    int64_t self = -1;
    double4 me = make_double4(0, 0, 0, 0);
    if (t < n) {
        const int64_t cid = targets[t];
        if (cid >= 0 && cid < ncells) {
            const int64_t leaf = cid / kCellsPerBlock;
            const int local = (int)(cid % kCellsPerBlock);
            const int f = internal_of_canon[leaf];
            self = (int64_t)f * kCellsPerBlock + morton9(local & 7, (local >> 3) & 7, local >> 6);
            me = cells[self];
        }
    }
    const double inv_L = 1.0 / L;
    double acc = 0.0;
    for (int64_t base = 0; base < ncells; base += 256) {
        __syncthreads();
        tile[threadIdx.x] = cells[base + threadIdx.x];  // ncells is a multiple of 512
        __syncthreads();
        double part = 0.0;
        for (int j = 0; j < 256; j++) {
            const double4 s = tile[j];
            if (s.w == 0.0) continue;
            double dx = me.x - s.x, dy = me.y - s.y, dz = me.z - s.z;
            dx -= L * rint(dx * inv_L);
            dy -= L * rint(dy * inv_L);
            dz -= L * rint(dz * inv_L);
            const double r2 = dx * dx + dy * dy + dz * dz;
            if (base + j != self) part += s.w / sqrt(r2);
            part += s.w * ewald_value_at(ew, dx, dy, dz);
        }
        acc += part;
    }
    if (self >= 0) phi[t] = -G * acc;
}

hipError_t launch_direct_periodic(const bh_grid *g, const bh_moments *m, const bh_ewald *e, const int64_t *targets,
                                  int64_t n, double G, double *out, hipStream_t s) {
    if (n == 0) return hipSuccess;
    EwaldView<double> ew{e->d_t64c, 1.0 / e->sp, e->sp, e->n, 1.0 / e->L, e->sp / e->L};
    hipLaunchKernelGGL(direct_periodic_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, targets, n,
                       m->d_cell64, g->n_cells, g->d_internal_of_canon, ew, e->L, G, out);
    return hipGetLastError();
}

}  // namespace bh
