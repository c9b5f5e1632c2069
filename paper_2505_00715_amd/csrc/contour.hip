// Points and weights of the gCQ integration contour (App. A), host code.
//
// The contour is the image of a horizontal line of the period rectangle of the
// Jacobi elliptic functions under the map gamma; only the largest and the
// smallest step sizes (and, for multi-stage Runge-Kutta methods, the spread
// of the stage eigenvalues) enter.  Complete elliptic integrals come from the
// arithmetic-geometric mean, the Jacobi functions of real argument from the
// descending Landen sequence of the same mean (Abramowitz & Stegun 17.6,
// 16.4), those of complex argument from the addition formulas (16.21).
#include <cmath>
#include <complex>

#include "internal.h"

namespace gcq {
namespace {

constexpr double PI = 3.14159265358979323846;

// K(m) = pi / (2 AGM(1, sqrt(m1))), parameter m = k^2 in [0, 1), m1 = 1 - m
// (passed separately, so that neither parameter loses digits to 1 - m)
double ellip_k(double m1) {
  double a = 1.0, b = std::sqrt(m1);
  for (int it = 0; it < 64 && std::fabs(a - b) > 1e-16 * a; ++it) {
    const double an = 0.5 * (a + b);
    b = std::sqrt(a * b);
    a = an;
  }
  return PI / (2.0 * a);
}

// sn, cn, dn of real u with parameter m in [0, 1): the AGM sequence
// a_{n+1} = (a_n + b_n)/2, b_{n+1} = sqrt(a_n b_n), c_{n+1} = (a_n - b_n)/2 down
// to c_N ~ 0, phi_N = 2^N a_N u, phi_{n-1} = (phi_n + asin(c_n sin(phi_n) / a_n)) / 2;
// sn = sin phi_0, cn = cos phi_0, and dn = sqrt(cn^2 + m1 sn^2) (= sqrt(1 - m sn^2)
// without its cancellation; the ratio cos phi_0 / cos(phi_1 - phi_0) is 0/0
// at u = K).
void ellip_j(double u, double m, double m1, double& sn, double& cn, double& dn) {
  if (m == 0.0) {
    sn = std::sin(u);
    cn = std::cos(u);
    dn = 1.0;
    return;
  }
  double a[40], c[40];
  a[0] = 1.0;
  double b = std::sqrt(m1);
  c[0] = std::sqrt(m);
  int n = 0;
  while (n < 38 && std::fabs(c[n]) > 1e-16 * a[n]) {
    a[n + 1] = 0.5 * (a[n] + b);
    c[n + 1] = 0.5 * (a[n] - b);
    b = std::sqrt(a[n] * b);
    ++n;
  }
  double phi = std::ldexp(a[n] * u, n);
  for (int j = n; j > 0; --j) phi = 0.5 * (phi + std::asin(c[j] * std::sin(phi) / a[j]));
  sn = std::sin(phi);
  cn = std::cos(phi);
  dn = std::sqrt(cn * cn + m1 * sn * sn);
}

// sn, cn, dn of x + i y (parameter m) from the real-argument functions at x
// (parameter m) and at y (parameter m1 = 1 - m)
void ellip_j_complex(double x, double y, double m, double m1, std::complex<double>& sn,
                     std::complex<double>& cn, std::complex<double>& dn) {
  double s, c, d, s1, c1, d1;
  ellip_j(x, m, m1, s, c, d);
  ellip_j(y, m1, m, s1, c1, d1);
  const double den = c1 * c1 + m * s * s * s1 * s1;
  sn = std::complex<double>(s * d1, c * d * s1 * c1) / den;
  cn = std::complex<double>(c * c1, -s * d * s1 * d1) / den;
  dn = std::complex<double>(d * c1 * d1, -m * s * c * s1) / den;
}

}  // namespace
}  // namespace gcq

using namespace gcq;

extern "C" GCQ_API int gcq_contour(int32_t n_points, double dt_min, double dt_max, double stage_ratio,
                                   gcq_c128* s, gcq_c128* w) {
  if (n_points < 1) return fail(GCQ_ERR_ARG, "n_points must be >= 1");
  if (!s || !w) return fail(GCQ_ERR_ARG, "s and w must not be NULL");
  if (!(dt_min > 0.0) || !(dt_max >= dt_min) || !std::isfinite(dt_max))
    return fail(GCQ_ERR_ARG, "need 0 < dt_min <= dt_max");
  if (!(stage_ratio >= 1.0) || !std::isfinite(stage_ratio))
    return fail(GCQ_ERR_ARG, "stage_ratio must be >= 1");
  const double q = stage_ratio * dt_max / dt_min;
  if (!(q > 1.0 + 1e-12))
    return fail(GCQ_ERR_ARG, "the step-size ratio q must exceed 1 (perturb it for constant steps)");
  const double r = std::sqrt(2.0 * q - 1.0);
  const double k = (q - r) / (q + r);
  const double m = k * k;
  const double m1 = (2.0 * r / (q + r)) * (1.0 + k);   // 1 - k^2 = (1 - k)(1 + k)
  const double K = ellip_k(m1), Kp = ellip_k(m);
  const double scale = 1.0 / (dt_min * (q - 1.0));
  const std::complex<double> wfac = std::complex<double>(0.0, -4.0 * K / (2.0 * PI * n_points));   // 4K / (2 pi i N_Q)
  for (int l = 1; l <= n_points; ++l) {
    const double x = -K + (l - 0.5) * 4.0 * K / n_points;
    std::complex<double> sn, cn, dn;
    ellip_j_complex(x, 0.5 * Kp, m, m1, sn, cn, dn);
    const std::complex<double> den = 1.0 / k - sn;
    const std::complex<double> g = scale * (r * (1.0 / k + sn) / den - 1.0);
    const std::complex<double> dg = scale * r * 2.0 * cn * dn / (k * den * den);
    const std::complex<double> ww = wfac * dg;
    s[l - 1] = {g.real(), g.imag()};
    w[l - 1] = {ww.real(), ww.imag()};
  }
  return GCQ_OK;
}

extern "C" GCQ_API int gcq_contour_points(int32_t n_steps, int32_t stages, int32_t* n_points) {
  if (!n_points) return fail(GCQ_ERR_ARG, "n_points must not be NULL");
  if (n_steps < 2 || stages < 1) return fail(GCQ_ERR_ARG, "need n_steps >= 2 and stages >= 1");
  const double lg = std::log(double(n_steps));
  const double half = 0.5 * n_steps * (stages == 1 ? lg : lg * lg);
  if (!(half < 1e9)) return fail(GCQ_ERR_ARG, "n_steps too large");
  *n_points = 2 * int32_t(std::llround(half));
  return GCQ_OK;
}
