// Forward gCQ convolution f = V * q with implicit Euler (Sec. 3: first step,
// eq. gCQ_xn, eq. gcq_formula) on the compressed operator of gcq_aca3d.
//
// Implicit Euler is the one-stage method A = (1), b = c = (1) (b^T A^{-1} = 1).
// With constant steps dt the current-step operator V(1/dt) is one more
// frequency of the set, so that each step is one product over the whole set
// [1/dt, s_1 .. s_NQ] followed by the sum of its columns:
//   f_n = V(1/dt) q_n + sum_l V(s_l) w_l x_{n-1}(s_l) / (1 - dt s_l),
//   x_{n-1}(s_l) = (x_{n-2}(s_l) + dt q_{n-1}) / (1 - dt s_l),  x_0 = 0.
// The state x (NQ x n, complex double) stays on the device; one kernel updates
// it and writes the product's input columns.  The sum over the set runs as the
// per-frequency product on the matrix cores (replayed as a graph) and a column
// sum, which is faster here than the eq.-product mode's frequency-weighted
// slices for a few dozen frequencies.
#include <chrono>
#include <cmath>
#include <complex>
#include <vector>

#include "internal.h"

namespace gcq {

// x_l <- (x_l + dt q_prev) / (1 - dt s_l) (when `advance`), then the product's
// columns: X[0] = q_cur, X[1 + l] = w_l x_l / (1 - dt s_l), for l < nq and the
// n triangles (vector-major, triangle order)
template <typename T>
__global__ void __launch_bounds__(256) gcq_columns(const double* __restrict__ q_prev,
                                                   const double* __restrict__ q_cur,
                                                   const double2* __restrict__ inv1m,
                                                   const double2* __restrict__ wl, int nq, int n,
                                                   double dt, int advance,
                                                   double2* __restrict__ x, cpx<T>* __restrict__ X) {
  const int64_t total = int64_t(nq + 1) * n;
  for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < total;
       e += int64_t(gridDim.x) * blockDim.x) {
    const int col = int(e / n), i = int(e % n);
    if (col == 0) {
      X[i] = {T(q_cur[i]), T(0)};
      continue;
    }
    const int l = col - 1;
    const double2 a = inv1m[l];   // 1 / (1 - dt s_l)
    double2 v = x[int64_t(l) * n + i];
    if (advance) {
      const double re = v.x + dt * q_prev[i], im = v.y;
      v = make_double2(re * a.x - im * a.y, re * a.y + im * a.x);
      x[int64_t(l) * n + i] = v;
    }
    // w_l v / (1 - dt s_l)
    const double2 b = wl[l];
    const double pr = v.x * a.x - v.y * a.y, pi = v.x * a.y + v.y * a.x;
    X[e] = {T(pr * b.x - pi * b.y), T(pr * b.y + pi * b.x)};
  }
}

// f = Re sum_k Y[k] (the columns are conjugate pairs, the sum is real)
template <typename T>
__global__ void __launch_bounds__(256) sum_columns_real(const cpx<T>* __restrict__ Y, int L, int n,
                                                        double* __restrict__ f) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    double acc = 0.0;
    for (int k = 0; k < L; ++k) acc += double(Y[int64_t(k) * n + i].re);
    f[i] = acc;
  }
}

}  // namespace gcq

using namespace gcq;

extern "C" GCQ_API int gcq_gcq_convolve(gcq_context* ctx, double dt, int32_t n_steps,
                                        const gcq_c128* w, int32_t precision, const double* Q,
                                        double* F) {
  if (!ctx) return fail(GCQ_ERR_ARG, "ctx is NULL");
  GCQ_NEED_DEVICE(ctx);
  if (!w || !Q || !F) return fail(GCQ_ERR_ARG, "w, Q and F must not be NULL");
  if (n_steps < 1) return fail(GCQ_ERR_ARG, "n_steps must be >= 1");
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(GCQ_ERR_ARG, "dt must be > 0");
  if (precision != GCQ_C128 && precision != GCQ_C64)
    return fail(GCQ_ERR_ARG, "unknown precision %d", precision);
  if (!ctx->F.valid || ctx->F.precision != precision)
    return fail(GCQ_ERR_STATE, "run gcq_aca3d at this precision first");
  const int L = ctx->L, n = ctx->n, nq = L - 1;
  if (L < 2) return fail(GCQ_ERR_STATE, "the frequency set needs 1/dt and at least one contour point");
  const std::complex<double> s0 = ctx->s[0];
  if (std::fabs(s0.real() - 1.0 / dt) > 1e-12 / dt || s0.imag() != 0.0)
    return fail(GCQ_ERR_STATE, "frequency 0 must be 1/dt (the current-step operator)");
  GCQ_HIP(hipSetDevice(ctx->device));
  std::vector<double2> inv1m(nq), wl(nq);
  for (int l = 0; l < nq; ++l) {
    const std::complex<double> d = 1.0 - dt * ctx->s[l + 1];
    if (std::abs(d) == 0.0) return fail(GCQ_ERR_ARG, "contour point %d equals 1/dt", l + 1);
    const std::complex<double> a = 1.0 / d;
    inv1m[l] = make_double2(a.real(), a.imag());
    wl[l] = make_double2(w[l].re, w[l].im);
  }
  hipStream_t st = ctx->stream;
  DevBuf d_inv, d_w, d_x, d_X, d_y;
  GCQ_TRY(upload(d_inv, inv1m, st));
  GCQ_TRY(upload(d_w, wl, st));
  GCQ_TRY(d_x.ensure(sizeof(double2) * size_t(nq) * n));
  GCQ_HIP(hipMemsetAsync(d_x.p, 0, sizeof(double2) * size_t(nq) * n, st));
  const size_t csz = csize(precision);
  GCQ_TRY(d_X.ensure(csz * size_t(L) * n));
  GCQ_TRY(d_y.ensure(csz * size_t(L) * n));
  const int grid = int(std::min<int64_t>((int64_t(L) * n + 255) / 256, int64_t(ctx->cus) * 16));
  // (each product synchronises on its own timing event, so the loop is timed
  // on the host clock)
  GCQ_HIP(hipStreamSynchronize(st));
  const auto t0 = std::chrono::steady_clock::now();
  for (int step = 0; step < n_steps; ++step) {
    const double* qp = step > 0 ? Q + int64_t(step - 1) * n : Q;
    const double* qc = Q + int64_t(step) * n;
    if (precision == GCQ_C128)
      hipLaunchKernelGGL(gcq_columns<double>, dim3(grid), dim3(256), 0, st, qp, qc, d_inv.as<double2>(),
                         d_w.as<double2>(), nq, n, dt, step > 0 ? 1 : 0, d_x.as<double2>(),
                         d_X.as<cpx<double>>());
    else
      hipLaunchKernelGGL(gcq_columns<float>, dim3(grid), dim3(256), 0, st, qp, qc, d_inv.as<double2>(),
                         d_w.as<double2>(), nq, n, dt, step > 0 ? 1 : 0, d_x.as<double2>(),
                         d_X.as<cpx<float>>());
    GCQ_HIP(hipGetLastError());
    GCQ_TRY(gcq_compressed_matvec(ctx, GCQ_PER_FREQUENCY, precision, d_X.p, d_y.p, L));
    const int g2 = std::min((n + 255) / 256, ctx->cus * 4);
    if (precision == GCQ_C128)
      hipLaunchKernelGGL(sum_columns_real<double>, dim3(g2), dim3(256), 0, st, d_y.as<cpx<double>>(), L,
                         n, F + int64_t(step) * n);
    else
      hipLaunchKernelGGL(sum_columns_real<float>, dim3(g2), dim3(256), 0, st, d_y.as<cpx<float>>(), L, n,
                         F + int64_t(step) * n);
    GCQ_HIP(hipGetLastError());
  }
  GCQ_HIP(hipStreamSynchronize(st));
  ctx->kernel_ms["gcq_convolve"] =
      std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  return GCQ_OK;
}

namespace gcq {

// B[0] = f - h (the system of frequency 0), B[k > 0] = 0
__global__ void __launch_bounds__(256) gcq_rhs(const double* __restrict__ f, const double* __restrict__ h,
                                               int L, int n, cpx<double>* __restrict__ B) {
  const int64_t total = int64_t(L) * n;
  for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < total;
       e += int64_t(gridDim.x) * blockDim.x)
    B[e] = e < n ? cpx<double>{f[e] - h[e], 0.0} : cpx<double>{0.0, 0.0};
}

__global__ void __launch_bounds__(256) gcq_take_real(const cpx<double>* __restrict__ X, int n,
                                                     double* __restrict__ q) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) q[i] = X[i].re;
}

}  // namespace gcq

extern "C" GCQ_API int gcq_gcq_solve(gcq_context* ctx, double dt, int32_t n_steps, const gcq_c128* w,
                                     int32_t precision, const double* F, double* Q, double rtol,
                                     int32_t max_iter, int32_t restart, int32_t* iters_max) {
  if (!ctx) return fail(GCQ_ERR_ARG, "ctx is NULL");
  GCQ_NEED_DEVICE(ctx);
  if (!w || !Q || !F) return fail(GCQ_ERR_ARG, "w, F and Q must not be NULL");
  if (n_steps < 1) return fail(GCQ_ERR_ARG, "n_steps must be >= 1");
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(GCQ_ERR_ARG, "dt must be > 0");
  if (precision != GCQ_C128 && precision != GCQ_C64)
    return fail(GCQ_ERR_ARG, "unknown precision %d", precision);
  if (!ctx->F.valid || ctx->F.precision != precision)
    return fail(GCQ_ERR_STATE, "run gcq_aca3d at this precision first");
  const int L = ctx->L, n = ctx->n, nq = L - 1;
  if (L < 2) return fail(GCQ_ERR_STATE, "the frequency set needs 1/dt and at least one contour point");
  const std::complex<double> s0 = ctx->s[0];
  if (std::fabs(s0.real() - 1.0 / dt) > 1e-12 / dt || s0.imag() != 0.0)
    return fail(GCQ_ERR_STATE, "frequency 0 must be 1/dt (the current-step operator)");
  GCQ_HIP(hipSetDevice(ctx->device));
  std::vector<double2> inv1m(nq), wl(nq);
  for (int l = 0; l < nq; ++l) {
    const std::complex<double> d = 1.0 - dt * ctx->s[l + 1];
    if (std::abs(d) == 0.0) return fail(GCQ_ERR_ARG, "contour point %d equals 1/dt", l + 1);
    const std::complex<double> a = 1.0 / d;
    inv1m[l] = make_double2(a.real(), a.imag());
    wl[l] = make_double2(w[l].re, w[l].im);
  }
  hipStream_t st = ctx->stream;
  const size_t csz = csize(precision);
  DevBuf d_inv, d_w, d_x, d_X, d_Y, d_zero, d_h, d_B, d_S;
  GCQ_TRY(upload(d_inv, inv1m, st));
  GCQ_TRY(upload(d_w, wl, st));
  GCQ_TRY(d_x.ensure(sizeof(double2) * size_t(nq) * n));
  GCQ_HIP(hipMemsetAsync(d_x.p, 0, sizeof(double2) * size_t(nq) * n, st));
  GCQ_TRY(d_X.ensure(csz * size_t(L) * n));
  GCQ_TRY(d_Y.ensure(csz * size_t(L) * n));
  GCQ_TRY(d_zero.ensure(sizeof(double) * n));
  GCQ_HIP(hipMemsetAsync(d_zero.p, 0, sizeof(double) * n, st));
  GCQ_TRY(d_h.ensure(sizeof(double) * n));
  GCQ_HIP(hipMemsetAsync(d_h.p, 0, sizeof(double) * n, st));
  GCQ_TRY(d_B.ensure(sizeof(cpx<double>) * size_t(L) * n));
  GCQ_TRY(d_S.ensure(sizeof(cpx<double>) * size_t(L) * n));
  const int grid = int(std::min<int64_t>((int64_t(L) * n + 255) / 256, int64_t(ctx->cus) * 16));
  const int g2 = std::min((n + 255) / 256, ctx->cus * 4);
  int itmax = 0;
  GCQ_HIP(hipStreamSynchronize(st));
  const auto t0 = std::chrono::steady_clock::now();
  for (int step = 0; step < n_steps; ++step) {
    if (step > 0) {
      // history of the earlier steps: the sum over the contour with the
      // current-step column left out
      const double* qp = Q + int64_t(step - 1) * n;
      if (precision == GCQ_C128)
        hipLaunchKernelGGL(gcq_columns<double>, dim3(grid), dim3(256), 0, st, qp, d_zero.as<double>(),
                           d_inv.as<double2>(), d_w.as<double2>(), nq, n, dt, 1, d_x.as<double2>(),
                           d_X.as<cpx<double>>());
      else
        hipLaunchKernelGGL(gcq_columns<float>, dim3(grid), dim3(256), 0, st, qp, d_zero.as<double>(),
                           d_inv.as<double2>(), d_w.as<double2>(), nq, n, dt, 1, d_x.as<double2>(),
                           d_X.as<cpx<float>>());
      GCQ_HIP(hipGetLastError());
      GCQ_TRY(gcq_compressed_matvec(ctx, GCQ_PER_FREQUENCY, precision, d_X.p, d_Y.p, L));
      if (precision == GCQ_C128)
        hipLaunchKernelGGL(sum_columns_real<double>, dim3(g2), dim3(256), 0, st, d_Y.as<cpx<double>>(), L,
                           n, d_h.as<double>());
      else
        hipLaunchKernelGGL(sum_columns_real<float>, dim3(g2), dim3(256), 0, st, d_Y.as<cpx<float>>(), L, n,
                           d_h.as<double>());
      GCQ_HIP(hipGetLastError());
    }
    // V(1/dt) q_n = f_n - history
    hipLaunchKernelGGL(gcq_rhs, dim3(grid), dim3(256), 0, st, F + int64_t(step) * n, d_h.as<double>(), L,
                       n, d_B.as<cpx<double>>());
    GCQ_HIP(hipGetLastError());
    gcq_solve_stats ss;
    GCQ_TRY(gcq_solve(ctx, d_B.p, d_S.p, rtol, max_iter, restart, precision, &ss));
    itmax = std::max(itmax, int(ss.iters_max));
    hipLaunchKernelGGL(gcq_take_real, dim3(g2), dim3(256), 0, st, d_S.as<cpx<double>>(), n,
                       Q + int64_t(step) * n);
    GCQ_HIP(hipGetLastError());
  }
  GCQ_HIP(hipStreamSynchronize(st));
  ctx->kernel_ms["gcq_solve"] =
      std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  if (iters_max) *iters_max = itmax;
  return GCQ_OK;
}
