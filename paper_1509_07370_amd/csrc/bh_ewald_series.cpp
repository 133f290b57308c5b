// Near-origin series of the smooth part D of the periodic Green's function
// (appendix "Periodic boundaries"), fitted when a table is created.
//
// D = psi - 1/|r| is smooth around the origin (its nearest singularities are
// the images at distance L), has the cube's symmetry and the Laplacian 4 pi /
// L^3 of the neutralising background.  In units of L (u = r / L) its series is
// therefore a polynomial in the symmetric functions of X = u_x^2, Y, Z:
//   D L = D0 + (2 pi / 3) e1 + [c1 e1^2 + c2 e2] + [c3 e1^3 + c4 e1 e2 + c5 e3]
//       + [c6 e1^4 + c7 e1^2 e2 + c8 e2^2 + c9 e1 e3] + O(|u|^10),
// e1 = X + Y + Z, e2 = XY + YZ + ZX, e3 = XYZ.  The fp32 periodic walks sum
// near tiles with it (no table rows for the pairs closest together); D0 and
// c1..c9 are fitted by least squares to the Ewald sums at points within
// kNearRadius, and the series is used only if it matches the sums at a second
// set of points to kNearTolerance.
#include <hip/hip_runtime.h>

#include <cmath>
#include <vector>

#include "bh_internal.h"

namespace bh {

namespace {

constexpr double kNearRadius = 0.15;     // in units of L
constexpr double kNearTolerance = 5e-8;  // largest |series - D L| allowed at the check points
constexpr int kFitSteps = 12;            // fit points: lattice of spacing kNearRadius / 12 in the octant ball

// the 9 fitted terms at u
void near_terms(const double *u, double *t) {
    const double X = u[0] * u[0], Y = u[1] * u[1], Z = u[2] * u[2];
    const double e1 = X + Y + Z, e2 = X * Y + Y * Z + Z * X, e3 = X * Y * Z;
    t[0] = e1 * e1;
    t[1] = e2;
    t[2] = e1 * e1 * e1;
    t[3] = e1 * e2;
    t[4] = e3;
    t[5] = e1 * e1 * e1 * e1;
    t[6] = e1 * e1 * e2;
    t[7] = e2 * e2;
    t[8] = e1 * e3;
}

double series_at(const double *c, const double *u) {
    double t[9];
    near_terms(u, t);
    double v = c[0] + c[1] * (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
    for (int k = 0; k < 9; k++) v += c[2 + k] * t[k];
    return v;
}

// Least squares min |A x - y| (rows m >= cols n, A row-major) by Householder
// QR on column-scaled A; false if a column is (numerically) dependent.
bool least_squares(std::vector<double> A, std::vector<double> y, int m, int n, double *x) {
    std::vector<double> scale(n, 0.0);
    for (int j = 0; j < n; j++) {
        for (int i = 0; i < m; i++) scale[j] = std::fmax(scale[j], std::fabs(A[i * n + j]));
        if (!(scale[j] > 0.0)) return false;
        for (int i = 0; i < m; i++) A[i * n + j] /= scale[j];
    }
    for (int j = 0; j < n; j++) {
        double norm = 0.0;
        for (int i = j; i < m; i++) norm += A[i * n + j] * A[i * n + j];
        norm = std::sqrt(norm);
        if (!(norm > 1e-12)) return false;
        const double alpha = A[j * n + j] > 0.0 ? -norm : norm;
        std::vector<double> v(m, 0.0);
        for (int i = j; i < m; i++) v[i] = A[i * n + j];
        v[j] -= alpha;
        double vv = 0.0;
        for (int i = j; i < m; i++) vv += v[i] * v[i];
        for (int k = j; k < n; k++) {
            double d = 0.0;
            for (int i = j; i < m; i++) d += v[i] * A[i * n + k];
            d = 2.0 * d / vv;
            for (int i = j; i < m; i++) A[i * n + k] -= d * v[i];
        }
        double d = 0.0;
        for (int i = j; i < m; i++) d += v[i] * y[i];
        d = 2.0 * d / vv;
        for (int i = j; i < m; i++) y[i] -= d * v[i];
    }
    for (int j = n - 1; j >= 0; j--) {
        double s = y[j];
        for (int k = j + 1; k < n; k++) s -= A[j * n + k] * x[k];
        x[j] = s / A[j * n + j];
    }
    for (int j = 0; j < n; j++) x[j] /= scale[j];
    return true;
}

}  // namespace

hipError_t fit_ewald_near_series(bh_ewald *e, hipStream_t s) {
    e->near_radius = 0.0;
    e->near_err = 0.0;
    // points in units of L: the origin, the fit lattice, then the check lattice (offset by half a step)
    const double h = kNearRadius / kFitSteps;
    std::vector<double> pts = {0.0, 0.0, 0.0};
    int n_fit = 0;
    for (int i = 0; i <= kFitSteps; i++)
        for (int j = 0; j <= kFitSteps; j++)
            for (int k = 0; k <= kFitSteps; k++) {
                const double u[3] = {i * h, j * h, k * h};
                if (u[0] * u[0] + u[1] * u[1] + u[2] * u[2] > kNearRadius * kNearRadius) continue;
                pts.insert(pts.end(), u, u + 3);
                n_fit++;
            }
    int n_check = 0;
    for (int i = 0; i < kFitSteps; i++)
        for (int j = 0; j < kFitSteps; j++)
            for (int k = 0; k < kFitSteps; k++) {
                const double u[3] = {(i + 0.5) * h, (j + 0.5) * h, (k + 0.5) * h};
                if (u[0] * u[0] + u[1] * u[1] + u[2] * u[2] > kNearRadius * kNearRadius) continue;
                pts.insert(pts.end(), u, u + 3);
                n_check++;
            }
    const int n = 1 + n_fit + n_check;
    double *d_pts = nullptr, *d_val = nullptr;
    hipError_t err = hipMalloc((void **)&d_pts, pts.size() * sizeof(double));
    if (err == hipSuccess) err = hipMalloc((void **)&d_val, n * sizeof(double));
    if (err == hipSuccess) err = hipMemcpyAsync(d_pts, pts.data(), pts.size() * sizeof(double), hipMemcpyHostToDevice, s);
    if (err == hipSuccess) err = launch_ewald_points(e->L, d_pts, n, d_val, s);
    std::vector<double> val(n);
    if (err == hipSuccess) err = hipMemcpyAsync(val.data(), d_val, n * sizeof(double), hipMemcpyDeviceToHost, s);
    if (err == hipSuccess) err = hipStreamSynchronize(s);
    if (d_pts) (void)hipFree(d_pts);
    if (d_val) (void)hipFree(d_val);
    if (err != hipSuccess) return err;
    // fit: D L - D0 - (2 pi / 3) e1 against the 9 terms
    double c[kEwaldNearTerms] = {val[0], 2.0 * 3.14159265358979323846 / 3.0};
    std::vector<double> A((size_t)n_fit * 9), y(n_fit);
    for (int q = 0; q < n_fit; q++) {
        const double *u = &pts[3 * (1 + q)];
        near_terms(u, &A[(size_t)q * 9]);
        y[q] = val[1 + q] - c[0] - c[1] * (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
    }
    if (!least_squares(A, y, n_fit, 9, c + 2)) return hipSuccess;  // the series stays unused
    double worst = 0.0;
    for (int q = 1; q < n; q++) worst = std::fmax(worst, std::fabs(series_at(c, &pts[3 * q]) - val[q]));
    for (int k = 0; k < kEwaldNearTerms; k++) e->near_coef[k] = c[k];
    e->near_err = worst;
    if (!(worst <= kNearTolerance)) return hipSuccess;
    float f[kEwaldNearTerms + 1];
    for (int k = 0; k < kEwaldNearTerms; k++) f[k] = (float)c[k];
    f[kEwaldNearTerms] = (float)(kNearRadius * kNearRadius);
    err = hipMemcpyAsync(e->d_near, f, sizeof(f), hipMemcpyHostToDevice, s);
    if (err == hipSuccess) err = hipStreamSynchronize(s);
    if (err == hipSuccess) e->near_radius = kNearRadius;
    return err;
}

}  // namespace bh
