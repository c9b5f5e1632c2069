// Forward gCQ convolution f = V * q with implicit Euler (Sec. 3: first step,
// eq. gCQ_xn, eq. gcq_formula) on the compressed operator of gcq_aca3d, and
// the solve for q with f given.
//
// Implicit Euler is the one-stage method A = (1), b = c = (1) (b^T A^{-1} = 1).
// The current-step operators V(1/dt_n) are frequencies of the set too: the set
// is [step points 1/dt (the distinct ones), contour points s_1 .. s_NQ], and
// each step is one product over the whole set followed by the sum of its
// columns:
//   f_n = V(1/dt_n) q_n + sum_l V(s_l) w_l x_{n-1}(s_l) / (1 - dt_n s_l),
//   x_{n-1}(s_l) = (x_{n-2}(s_l) + dt_{n-1} q_{n-1}) / (1 - dt_{n-1} s_l),  x_0 = 0.
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

// complex a / b
__device__ inline double2 zdiv(double2 a, double2 b) {
  const double d = b.x * b.x + b.y * b.y;
  return make_double2((a.x * b.x + a.y * b.y) / d, (a.y * b.x - a.x * b.y) / d);
}

// The product's columns for one step, n triangles each (vector-major, triangle
// order): the np step-point columns hold q_cur in column kcur and 0 elsewhere;
// contour column np + l first advances x_l <- (x_l + dt_prev q_prev) /
// (1 - dt_prev s_l) (when `advance`), then holds w_l x_l / (1 - dt_cur s_l).
template <typename T>
__global__ void __launch_bounds__(256) gcq_columns(const double* __restrict__ q_prev,
                                                   const double* __restrict__ q_cur,
                                                   const double2* __restrict__ sl,
                                                   const double2* __restrict__ wl, int np, int kcur,
                                                   int nq, int n, double dt_prev, double dt_cur,
                                                   int advance, double2* __restrict__ x,
                                                   cpx<T>* __restrict__ X) {
  const int64_t total = int64_t(np + nq) * n;
  for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < total;
       e += int64_t(gridDim.x) * blockDim.x) {
    const int col = int(e / n), i = int(e % n);
    if (col < np) {
      X[e] = {col == kcur ? T(q_cur[i]) : T(0), T(0)};
      continue;
    }
    const int l = col - np;
    const double2 s = sl[l];
    double2 v = x[int64_t(l) * n + i];
    if (advance) {
      v = zdiv(make_double2(v.x + dt_prev * q_prev[i], v.y),
               make_double2(1.0 - dt_prev * s.x, -dt_prev * s.y));
      x[int64_t(l) * n + i] = v;
    }
    const double2 b = wl[l];
    const double2 u = make_double2(v.x * b.x - v.y * b.y, v.x * b.y + v.y * b.x);   // w_l x_l
    const double2 r = zdiv(u, make_double2(1.0 - dt_cur * s.x, -dt_cur * s.y));
    X[e] = {T(r.x), T(r.y)};
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

namespace gcq {

// B[kcur] = f - h (the system of the current step's point), other columns 0
__global__ void __launch_bounds__(256) gcq_rhs(const double* __restrict__ f, const double* __restrict__ h,
                                               int kcur, int L, int n, cpx<double>* __restrict__ B) {
  const int64_t total = int64_t(L) * n;
  for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < total;
       e += int64_t(gridDim.x) * blockDim.x) {
    const int col = int(e / n), i = int(e % n);
    B[e] = col == kcur ? cpx<double>{f[i] - h[i], 0.0} : cpx<double>{0.0, 0.0};
  }
}

__global__ void __launch_bounds__(256) gcq_take_real(const cpx<double>* __restrict__ X, int n,
                                                     double* __restrict__ q) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) q[i] = X[i].re;
}

// checks shared by the two entry points; kstep[n] = the frequency 1/dt_n,
// contour points and weights to the device, state x zeroed
struct GcqRun {
  int L = 0, n = 0, np = 0, nq = 0;
  std::vector<int> kstep;
  DevBuf d_s, d_w, d_x, d_X, d_Y;
};

static int gcq_prepare(gcq_context* ctx, const double* dt, int n_steps, int n_step_points,
                       const gcq_c128* w, int precision, GcqRun& R) {
  if (!ctx) return fail(GCQ_ERR_ARG, "ctx is NULL");
  GCQ_NEED_DEVICE(ctx);
  if (!dt || !w) return fail(GCQ_ERR_ARG, "dt and w must not be NULL");
  if (n_steps < 1) return fail(GCQ_ERR_ARG, "n_steps must be >= 1");
  if (precision != GCQ_C128 && precision != GCQ_C64)
    return fail(GCQ_ERR_ARG, "unknown precision %d", precision);
  if (!ctx->F.valid || ctx->F.precision != precision)
    return fail(GCQ_ERR_STATE, "run gcq_aca3d at this precision first");
  R.L = ctx->L;
  R.n = ctx->n;
  R.np = n_step_points;
  R.nq = R.L - R.np;
  if (R.np < 1 || R.nq < 1)
    return fail(GCQ_ERR_ARG, "need 1 <= n_step_points < n_freq (step points, then contour points)");
  R.kstep.assign(n_steps, -1);
  for (int st = 0; st < n_steps; ++st) {
    if (!(dt[st] > 0.0) || !std::isfinite(dt[st])) return fail(GCQ_ERR_ARG, "dt[%d] must be > 0", st);
    for (int k = 0; k < R.np && R.kstep[st] < 0; ++k)
      if (ctx->s[k].imag() == 0.0 && std::fabs(ctx->s[k].real() - 1.0 / dt[st]) <= 1e-12 / dt[st])
        R.kstep[st] = k;
    if (R.kstep[st] < 0)
      return fail(GCQ_ERR_STATE, "no step-point frequency equals 1/dt of step %d", st);
  }
  GCQ_HIP(hipSetDevice(ctx->device));
  std::vector<double2> sl(R.nq), wl(R.nq);
  for (int l = 0; l < R.nq; ++l) {
    const std::complex<double> z = ctx->s[R.np + l];
    sl[l] = make_double2(z.real(), z.imag());
    wl[l] = make_double2(w[l].re, w[l].im);
  }
  hipStream_t st = ctx->stream;
  GCQ_TRY(upload(R.d_s, sl, st));
  GCQ_TRY(upload(R.d_w, wl, st));
  GCQ_TRY(R.d_x.ensure(sizeof(double2) * size_t(R.nq) * R.n));
  GCQ_HIP(hipMemsetAsync(R.d_x.p, 0, sizeof(double2) * size_t(R.nq) * R.n, st));
  const size_t csz = csize(precision);
  GCQ_TRY(R.d_X.ensure(csz * size_t(R.L) * R.n));
  GCQ_TRY(R.d_Y.ensure(csz * size_t(R.L) * R.n));
  return GCQ_OK;
}

// one product over the set and the column sum into h (length n)
static int gcq_apply_step(gcq_context* ctx, GcqRun& R, int precision, const double* q_prev,
                          const double* q_cur, int kcur, double dt_prev, double dt_cur, int advance,
                          double* h) {
  hipStream_t st = ctx->stream;
  const int grid = int(std::min<int64_t>((int64_t(R.L) * R.n + 255) / 256, int64_t(ctx->cus) * 16));
  const int g2 = std::min((R.n + 255) / 256, ctx->cus * 4);
  if (precision == GCQ_C128)
    hipLaunchKernelGGL(gcq_columns<double>, dim3(grid), dim3(256), 0, st, q_prev, q_cur, R.d_s.as<double2>(),
                       R.d_w.as<double2>(), R.np, kcur, R.nq, R.n, dt_prev, dt_cur, advance,
                       R.d_x.as<double2>(), R.d_X.as<cpx<double>>());
  else
    hipLaunchKernelGGL(gcq_columns<float>, dim3(grid), dim3(256), 0, st, q_prev, q_cur, R.d_s.as<double2>(),
                       R.d_w.as<double2>(), R.np, kcur, R.nq, R.n, dt_prev, dt_cur, advance,
                       R.d_x.as<double2>(), R.d_X.as<cpx<float>>());
  GCQ_HIP(hipGetLastError());
  GCQ_TRY(gcq_compressed_matvec(ctx, GCQ_PER_FREQUENCY, precision, R.d_X.p, R.d_Y.p, R.L));
  if (precision == GCQ_C128)
    hipLaunchKernelGGL(sum_columns_real<double>, dim3(g2), dim3(256), 0, st, R.d_Y.as<cpx<double>>(), R.L,
                       R.n, h);
  else
    hipLaunchKernelGGL(sum_columns_real<float>, dim3(g2), dim3(256), 0, st, R.d_Y.as<cpx<float>>(), R.L, R.n,
                       h);
  GCQ_HIP(hipGetLastError());
  return GCQ_OK;
}

}  // namespace gcq

extern "C" GCQ_API int gcq_gcq_convolve(gcq_context* ctx, const double* dt, int32_t n_steps,
                                        int32_t n_step_points, const gcq_c128* w, int32_t precision,
                                        const double* Q, double* F) {
  GcqRun R;
  GCQ_TRY(gcq_prepare(ctx, dt, n_steps, n_step_points, w, precision, R));
  if (!Q || !F) return fail(GCQ_ERR_ARG, "Q and F must not be NULL");
  const int n = R.n;
  GCQ_HIP(hipStreamSynchronize(ctx->stream));
  const auto t0 = std::chrono::steady_clock::now();
  for (int step = 0; step < n_steps; ++step) {
    const double* qp = step > 0 ? Q + int64_t(step - 1) * n : Q;
    GCQ_TRY(gcq_apply_step(ctx, R, precision, qp, Q + int64_t(step) * n, R.kstep[step],
                           step > 0 ? dt[step - 1] : 0.0, dt[step], step > 0 ? 1 : 0,
                           F + int64_t(step) * n));
  }
  GCQ_HIP(hipStreamSynchronize(ctx->stream));
  ctx->kernel_ms["gcq_convolve"] =
      std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  return GCQ_OK;
}

extern "C" GCQ_API int gcq_gcq_solve(gcq_context* ctx, const double* dt, int32_t n_steps,
                                     int32_t n_step_points, const gcq_c128* w, int32_t precision,
                                     const double* F, double* Q, double rtol, int32_t max_iter,
                                     int32_t restart, int32_t* iters_max) {
  GcqRun R;
  GCQ_TRY(gcq_prepare(ctx, dt, n_steps, n_step_points, w, precision, R));
  if (!Q || !F) return fail(GCQ_ERR_ARG, "F and Q must not be NULL");
  const int n = R.n, L = R.L;
  hipStream_t st = ctx->stream;
  DevBuf d_zero, d_h, d_B, d_S;
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
    // history of the earlier steps: the contour sum, no step-point column
    if (step > 0)
      GCQ_TRY(gcq_apply_step(ctx, R, precision, Q + int64_t(step - 1) * n, d_zero.as<double>(), -1,
                             dt[step - 1], dt[step], 1, d_h.as<double>()));
    // V(1/dt_n) q_n = f_n - history
    const int k = R.kstep[step];
    hipLaunchKernelGGL(gcq_rhs, dim3(grid), dim3(256), 0, st, F + int64_t(step) * n, d_h.as<double>(), k, L,
                       n, d_B.as<cpx<double>>());
    GCQ_HIP(hipGetLastError());
    gcq_solve_stats ss;
    GCQ_TRY(gcq_solve(ctx, d_B.p, d_S.p, rtol, max_iter, restart, precision, &ss));
    itmax = std::max(itmax, int(ss.iters_max));
    hipLaunchKernelGGL(gcq_take_real, dim3(g2), dim3(256), 0, st, d_S.as<cpx<double>>() + int64_t(k) * n, n,
                       Q + int64_t(step) * n);
    GCQ_HIP(hipGetLastError());
  }
  GCQ_HIP(hipStreamSynchronize(st));
  ctx->kernel_ms["gcq_solve"] =
      std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  if (iters_max) *iters_max = itmax;
  return GCQ_OK;
}
