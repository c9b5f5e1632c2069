// gCQ time stepping (Sec. 3: the first step, eq. gCQ_xn, eq. gcq_formula) on
// the compressed operator of gcq_aca3d: the forward convolution f = V * q for
// a given density and the solve for the density with f given, for an m-stage
// Runge-Kutta method (c | A, b^T) with b^T A^{-1} = (0, .., 0, 1) and variable
// steps.  Quantities per node carry the m stage values; implicit Euler is
// m = 1, A = (1).
//
// The set of frequencies is [step points, contour points s_1 .. s_NQ]: the
// step points are the values lam_e / dt (lam_e the eigenvalues of A^{-1}) for
// every distinct step dt, so that V((dt A)^{-1}) = P diag(V(lam_e / dt)) P^{-1}
// (A^{-1} = P diag(lam) P^{-1}) is a combination of product columns.  Per
// step n, with M_l(dt) = (I - dt s_l A)^{-1}:
//   x_{n-1}(s_l) = M_l(dt_{n-1}) ((b^T A^{-1} x_{n-2}(s_l)) 1 + dt_{n-1} A q_{n-1}),
//   f_n = V((dt_n A)^{-1}) q_n + sum_l V(s_l) w_l (b^T A^{-1} x_{n-1}(s_l)) M_l(dt_n) 1.
// Only the last stage of x enters (b^T A^{-1} picks it), so the state is one
// complex value per contour point and node, kept on the device:
//   x_l <- r_l x_l + sum_j g_lj (q_{n-1})_j,  r_l = (M_l 1)_m,  g_l = dt (M_l A)_{m,:}.
// Stage i of f_n is one product over the whole set (step-point columns
// sum_j P_ie P^{-1}_ej (q_n)_j, contour columns w_l (M_l(dt_n) 1)_i x_l) and
// the sum of its columns.  The product runs per frequency on the matrix cores
// (replayed as a graph), which is faster here than the eq.-product mode's
// frequency-weighted slices for a few dozen frequencies.  The m x m algebra
// (the eigendecomposition of A^{-1}, the M_l of every step) is host work done
// once per call; its coefficients go to the device in one copy.
#include <chrono>
#include <cmath>
#include <complex>
#include <vector>

#include "internal.h"

namespace gcq {

using zd = std::complex<double>;
constexpr int GCQ_MAX_STAGES = 4;

// ---- host: small dense complex algebra (m <= 4) --------------------------------
// solve M X = B (M m x m, B m x k, row-major) by Gaussian elimination with
// partial pivoting; false when a pivot vanishes
static bool zsolve(std::vector<zd> M, std::vector<zd>& B, int m, int k) {
  for (int c = 0; c < m; ++c) {
    int p = c;
    for (int r = c + 1; r < m; ++r)
      if (std::abs(M[r * m + c]) > std::abs(M[p * m + c])) p = r;
    if (std::abs(M[p * m + c]) == 0.0) return false;
    if (p != c) {
      for (int j = 0; j < m; ++j) std::swap(M[c * m + j], M[p * m + j]);
      for (int j = 0; j < k; ++j) std::swap(B[c * k + j], B[p * k + j]);
    }
    for (int r = c + 1; r < m; ++r) {
      const zd f = M[r * m + c] / M[c * m + c];
      for (int j = c; j < m; ++j) M[r * m + j] -= f * M[c * m + j];
      for (int j = 0; j < k; ++j) B[r * k + j] -= f * B[c * k + j];
    }
  }
  for (int c = m - 1; c >= 0; --c)
    for (int j = 0; j < k; ++j) {
      zd acc = B[c * k + j];
      for (int i = c + 1; i < m; ++i) acc -= M[c * m + i] * B[i * k + j];
      B[c * k + j] = acc / M[c * m + c];
    }
  return true;
}

// T = P diag(lam) P^{-1} for a real m x m matrix T (row-major): the
// characteristic polynomial by the Faddeev-LeVerrier recursion, its roots by
// the Durand-Kerner (Weierstrass) iteration, the eigenvectors by inverse
// iteration.  False when the result does not reproduce T P = P diag(lam).
static bool eigen_small(const std::vector<double>& T, int m, std::vector<zd>& lam, std::vector<zd>& P,
                        std::vector<zd>& Pinv) {
  // p(x) = x^m + c_1 x^{m-1} + ... + c_m;  B_k = T B_{k-1} + c_{k-1} I,  c_k = -tr(T B_k) / k
  std::vector<double> c(m + 1, 0.0), Bk(m * m, 0.0), TB(m * m);
  c[0] = 1.0;
  for (int k = 1; k <= m; ++k) {
    for (int i = 0; i < m; ++i)
      for (int j = 0; j < m; ++j) {
        double acc = 0.0;
        for (int l = 0; l < m; ++l) acc += T[i * m + l] * Bk[l * m + j];
        TB[i * m + j] = acc + (i == j ? c[k - 1] : 0.0);
      }
    Bk = TB;
    double tr = 0.0;
    for (int i = 0; i < m; ++i)
      for (int l = 0; l < m; ++l) tr += T[i * m + l] * Bk[l * m + i];
    c[k] = -tr / k;
  }
  auto poly = [&](zd x) {
    zd v = 1.0;
    for (int k = 1; k <= m; ++k) v = v * x + c[k];
    return v;
  };
  double scale = 1.0;   // bound on the roots' size
  for (int k = 1; k <= m; ++k) scale = std::max(scale, std::pow(std::fabs(c[k]), 1.0 / k));
  lam.assign(m, 0.0);
  for (int e = 0; e < m; ++e) lam[e] = scale * std::pow(zd(0.4, 0.9), e);
  for (int it = 0; it < 500; ++it) {
    double delta = 0.0;
    for (int e = 0; e < m; ++e) {
      zd den = 1.0;
      for (int f = 0; f < m; ++f)
        if (f != e) den *= lam[e] - lam[f];
      if (std::abs(den) == 0.0) return false;
      const zd step = poly(lam[e]) / den;
      lam[e] -= step;
      delta = std::max(delta, std::abs(step) / std::max(1.0, std::abs(lam[e])));
    }
    if (delta < 1e-16) break;
  }
  P.assign(m * m, 0.0);
  for (int e = 0; e < m; ++e) {
    std::vector<zd> M(m * m);
    const zd shift = lam[e] * (1.0 + 1e-13) + 1e-14 * scale;
    for (int i = 0; i < m; ++i)
      for (int j = 0; j < m; ++j) M[i * m + j] = T[i * m + j] - (i == j ? shift : 0.0);
    std::vector<zd> v(m);
    for (int i = 0; i < m; ++i) v[i] = zd(1.0 + 0.1 * i, 0.05 * i);
    for (int it = 0; it < 3; ++it) {
      if (!zsolve(M, v, m, 1)) return false;
      double nv = 0.0;
      for (int i = 0; i < m; ++i) nv += std::norm(v[i]);
      nv = std::sqrt(nv);
      if (!(nv > 0.0) || !std::isfinite(nv)) return false;
      for (int i = 0; i < m; ++i) v[i] /= nv;
    }
    for (int i = 0; i < m; ++i) P[i * m + e] = v[i];
  }
  Pinv.assign(m * m, 0.0);
  for (int i = 0; i < m; ++i) Pinv[i * m + i] = 1.0;
  if (!zsolve(P, Pinv, m, m)) return false;
  double err = 0.0, tn = 0.0, pin = 0.0;
  for (int i = 0; i < m; ++i)
    for (int e = 0; e < m; ++e) {
      zd acc = 0.0;
      for (int l = 0; l < m; ++l) acc += T[i * m + l] * P[l * m + e];
      err = std::max(err, std::abs(acc - P[i * m + e] * lam[e]));
      tn = std::max(tn, std::fabs(T[i * m + e]));
      pin = std::max(pin, std::abs(Pinv[i * m + e]));
    }
  return err <= 1e-9 * std::max(tn, 1.0) && pin < 1e8;   // 1e8: P nearly singular (defective A^{-1})
}

// ---- device kernels --------------------------------------------------------------
// state x_l <- r_l x_l + sum_j g_lj q_prev[j]   (x: nq x n complex; q_prev: m x n)
__global__ void __launch_bounds__(256) gcq_state(const double* __restrict__ q_prev, int m, int nq, int n,
                                                 const double2* __restrict__ r, const double2* __restrict__ g,
                                                 double2* __restrict__ x) {
  const int64_t total = int64_t(nq) * n;
  for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < total;
       e += int64_t(gridDim.x) * blockDim.x) {
    const int l = int(e / n), i = int(e % n);
    const double2 rl = r[l], v = x[e];
    double re = rl.x * v.x - rl.y * v.y, im = rl.x * v.y + rl.y * v.x;
    for (int j = 0; j < m; ++j) {
      const double2 gj = g[l * m + j];
      const double qj = q_prev[int64_t(j) * n + i];
      re += gj.x * qj;
      im += gj.y * qj;
    }
    x[e] = make_double2(re, im);
  }
}

// The product's columns for stage i of a step, n triangles each (vector-major,
// triangle order): step-point column k holds sum_j tq[e][j] q_cur[j] with
// e = ce[k] (ce[k] < 0 or no q_cur: zero), contour column np + l holds cl[l] x_l.
template <typename T>
__global__ void __launch_bounds__(256) gcq_columns(const double* __restrict__ q_cur, int m, int np, int nq,
                                                   int n, const int* __restrict__ ce,
                                                   const double2* __restrict__ tq,
                                                   const double2* __restrict__ cl,
                                                   const double2* __restrict__ x, cpx<T>* __restrict__ X) {
  const int64_t total = int64_t(np + nq) * n;
  for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < total;
       e += int64_t(gridDim.x) * blockDim.x) {
    const int col = int(e / n), i = int(e % n);
    if (col < np) {
      const int ee = ce[col];
      double re = 0.0, im = 0.0;
      if (ee >= 0 && q_cur)
        for (int j = 0; j < m; ++j) {
          const double2 t = tq[ee * m + j];
          const double qj = q_cur[int64_t(j) * n + i];
          re += t.x * qj;
          im += t.y * qj;
        }
      X[e] = {T(re), T(im)};
      continue;
    }
    const int l = col - np;
    const double2 c = cl[l], v = x[int64_t(l) * n + i];
    X[e] = {T(c.x * v.x - c.y * v.y), T(c.x * v.y + c.y * v.x)};
  }
}

// f = Re sum_k Y[k] (the stage value is real: conjugate columns pair up)
template <typename T>
__global__ void __launch_bounds__(256) sum_columns_real(const cpx<T>* __restrict__ Y, int L, int n,
                                                        double* __restrict__ f) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    double acc = 0.0;
    for (int k = 0; k < L; ++k) acc += double(Y[int64_t(k) * n + i].re);
    f[i] = acc;
  }
}

// right-hand sides of the decoupled systems of one step: column k = ke[e] holds
// sum_j P^{-1}_ej (f_j - h_j), every other column 0
__global__ void __launch_bounds__(256) gcq_rhs(const double* __restrict__ f, const double* __restrict__ h,
                                               int m, int np, int L, int n, const int* __restrict__ ce,
                                               const double2* __restrict__ pinv, cpx<double>* __restrict__ B) {
  const int64_t total = int64_t(L) * n;
  for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < total;
       e += int64_t(gridDim.x) * blockDim.x) {
    const int col = int(e / n), i = int(e % n);
    const int ee = col < np ? ce[col] : -1;
    double re = 0.0, im = 0.0;
    if (ee >= 0)
      for (int j = 0; j < m; ++j) {
        const double2 t = pinv[ee * m + j];
        const double rj = f[int64_t(j) * n + i] - h[int64_t(j) * n + i];
        re += t.x * rj;
        im += t.y * rj;
      }
    B[e] = {re, im};
  }
}

// stage values q_i = Re sum_e P_ie S[ke[e]]
__global__ void __launch_bounds__(256) gcq_take(const cpx<double>* __restrict__ S, int m, int n,
                                                const int* __restrict__ ke, const double2* __restrict__ Pm,
                                                double* __restrict__ q) {
  const int64_t total = int64_t(m) * n;
  for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < total;
       e += int64_t(gridDim.x) * blockDim.x) {
    const int i = int(e / n), v = int(e % n);
    double acc = 0.0;
    for (int ee = 0; ee < m; ++ee) {
      const double2 p = Pm[i * m + ee];
      const cpx<double> y = S[int64_t(ke[ee]) * n + v];
      acc += p.x * y.re - p.y * y.im;
    }
    q[e] = acc;
  }
}

// ---- host driver ------------------------------------------------------------------
// Coefficients of every step in one device block.  Per step (double2 units):
// r (nq), g (nq x m), c (m x nq); then once: tq (m x m x m), pinv, P (m x m).
// Per step (ints): ce (np), ke (m).
struct GcqRun {
  int L = 0, n = 0, m = 0, np = 0, nq = 0, n_steps = 0;
  size_t step_d = 0, step_i = 0;      // per-step block sizes
  std::vector<double2> hcoef;         // host copies (alive until the call returns)
  std::vector<int> hidx;
  DevBuf d_coef, d_idx, d_x, d_X, d_Y;
  const double2* r(int st) const { return d_coef.as<double2>() + st * step_d; }
  const double2* g(int st) const { return r(st) + nq; }
  const double2* c(int st) const { return g(st) + size_t(nq) * m; }
  const double2* tq() const { return d_coef.as<double2>() + n_steps * step_d; }
  const double2* pinv() const { return tq() + m * m * m; }
  const double2* P() const { return pinv() + m * m; }
  const int* ce(int st) const { return d_idx.as<int>() + st * step_i; }
  const int* ke(int st) const { return ce(st) + np; }
};

static inline double2 d2(zd z) { return make_double2(z.real(), z.imag()); }

// checks shared by the entry points, the method's algebra and every step's
// coefficients, uploaded; state x zeroed
static int gcq_prepare(gcq_context* ctx, const double* A, int m, const double* dt, int n_steps,
                       int n_step_points, const gcq_c128* w, int precision, GcqRun& R) {
  if (!ctx) return fail(GCQ_ERR_ARG, "ctx is NULL");
  GCQ_NEED_DEVICE(ctx);
  if (!A || !dt || !w) return fail(GCQ_ERR_ARG, "A, dt and w must not be NULL");
  if (m < 1 || m > GCQ_MAX_STAGES) return fail(GCQ_ERR_ARG, "m must be in 1..%d", GCQ_MAX_STAGES);
  if (n_steps < 1) return fail(GCQ_ERR_ARG, "n_steps must be >= 1");
  if (precision != GCQ_C128 && precision != GCQ_C64)
    return fail(GCQ_ERR_ARG, "unknown precision %d", precision);
  if (!ctx->F.valid || ctx->F.precision != precision)
    return fail(GCQ_ERR_STATE, "run gcq_aca3d at this precision first");
  if (ctx->F.near_only)
    return fail(GCQ_ERR_STATE, "the 3D operator holds only the near field of the FMM-based variant");
  R.L = ctx->L;
  R.n = ctx->n;
  R.m = m;
  R.np = n_step_points;
  R.nq = R.L - R.np;
  R.n_steps = n_steps;
  if (R.np < m || R.nq < 1)
    return fail(GCQ_ERR_ARG, "need m <= n_step_points < n_freq (step points, then contour points)");
  for (int i = 0; i < m * m; ++i)
    if (!std::isfinite(A[i])) return fail(GCQ_ERR_ARG, "A holds a non-finite entry");
  // A^{-1} = P diag(lam) P^{-1}
  std::vector<zd> Ai(m * m, 0.0), Az(m * m);
  for (int i = 0; i < m; ++i) Ai[i * m + i] = 1.0;
  for (int i = 0; i < m * m; ++i) Az[i] = A[i];
  if (!zsolve(Az, Ai, m, m)) return fail(GCQ_ERR_ARG, "A is singular");
  std::vector<double> Ar(m * m);
  for (int i = 0; i < m * m; ++i) Ar[i] = Ai[i].real();
  std::vector<zd> lam, P, Pinv;
  if (!eigen_small(Ar, m, lam, P, Pinv)) return fail(GCQ_ERR_NUMERIC, "A^{-1} is not diagonalisable");
  R.step_d = size_t(R.nq) * (1 + 2 * m);
  R.step_i = size_t(R.np) + m;
  R.hcoef.assign(n_steps * R.step_d + size_t(m) * m * m + 2 * m * m, make_double2(0, 0));
  R.hidx.assign(n_steps * R.step_i, -1);
  for (int st = 0; st < n_steps; ++st) {
    if (!(dt[st] > 0.0) || !std::isfinite(dt[st])) return fail(GCQ_ERR_ARG, "dt[%d] must be > 0", st);
    int* ce = R.hidx.data() + st * R.step_i;
    int* ke = ce + R.np;
    for (int e = 0; e < m; ++e) {
      const zd z = lam[e] / dt[st];
      ke[e] = -1;
      for (int k = 0; k < R.np && ke[e] < 0; ++k)
        if (std::abs(ctx->s[k] - z) <= 1e-10 * std::abs(z)) ke[e] = k;
      if (ke[e] < 0) return fail(GCQ_ERR_STATE, "step %d: no step-point frequency equals lambda_%d(A^{-1})/dt", st, e);
      if (ce[ke[e]] >= 0) return fail(GCQ_ERR_NUMERIC, "A^{-1} has a repeated eigenvalue");
      ce[ke[e]] = e;
    }
    // r, g of the update into this step (dt_{n-1}), c of this step (dt_n)
    double2* r = R.hcoef.data() + st * R.step_d;
    double2* g = r + R.nq;
    double2* c = g + size_t(R.nq) * m;
    for (int l = 0; l < R.nq; ++l) {
      const zd s = ctx->s[R.np + l];
      std::vector<zd> M(m * m);
      if (st > 0) {
        const double h = dt[st - 1];
        std::vector<zd> E(m * m, 0.0);
        for (int i = 0; i < m; ++i) E[i * m + i] = 1.0;
        for (int i = 0; i < m; ++i)
          for (int j = 0; j < m; ++j) M[i * m + j] = (i == j ? 1.0 : 0.0) - h * s * A[i * m + j];
        if (!zsolve(M, E, m, m)) return fail(GCQ_ERR_NUMERIC, "I - dt s_%d A is singular", l);
        zd rr = 0.0;
        for (int j = 0; j < m; ++j) rr += E[(m - 1) * m + j];
        r[l] = d2(rr);
        for (int j = 0; j < m; ++j) {
          zd acc = 0.0;
          for (int k = 0; k < m; ++k) acc += E[(m - 1) * m + k] * A[k * m + j];
          g[size_t(l) * m + j] = d2(h * acc);
        }
      }
      std::vector<zd> u(m, 1.0);
      for (int i = 0; i < m; ++i)
        for (int j = 0; j < m; ++j) M[i * m + j] = (i == j ? 1.0 : 0.0) - dt[st] * s * A[i * m + j];
      if (!zsolve(M, u, m, 1)) return fail(GCQ_ERR_NUMERIC, "I - dt s_%d A is singular", l);
      const zd wl(w[l].re, w[l].im);
      for (int i = 0; i < m; ++i) c[size_t(i) * R.nq + l] = d2(wl * u[i]);
    }
  }
  double2* tq = R.hcoef.data() + n_steps * R.step_d;
  for (int i = 0; i < m; ++i)
    for (int e = 0; e < m; ++e)
      for (int j = 0; j < m; ++j) tq[(i * m + e) * m + j] = d2(P[i * m + e] * Pinv[e * m + j]);
  for (int i = 0; i < m * m; ++i) {
    tq[m * m * m + i] = d2(Pinv[i]);
    tq[m * m * m + m * m + i] = d2(P[i]);
  }
  GCQ_HIP(hipSetDevice(ctx->device));
  hipStream_t st = ctx->stream;
  GCQ_TRY(upload(R.d_coef, R.hcoef, st));
  GCQ_TRY(upload(R.d_idx, R.hidx, st));
  GCQ_TRY(R.d_x.ensure(sizeof(double2) * size_t(R.nq) * R.n));
  GCQ_HIP(hipMemsetAsync(R.d_x.p, 0, sizeof(double2) * size_t(R.nq) * R.n, st));
  const size_t csz = csize(precision);
  GCQ_TRY(R.d_X.ensure(csz * size_t(R.L) * R.n));
  GCQ_TRY(R.d_Y.ensure(csz * size_t(R.L) * R.n));
  GCQ_HIP(hipStreamSynchronize(st));   // the host coefficient copies are free after this
  return GCQ_OK;
}

// stage i of step `step`: columns, one product over the set, column sum into out
static int stage_product(gcq_context* ctx, GcqRun& R, int precision, int step, const double* q_cur, int i,
                         double* out) {
  hipStream_t st = ctx->stream;
  const int grid = int(std::min<int64_t>((int64_t(R.L) * R.n + 255) / 256, int64_t(ctx->cus) * 16));
  const int g2 = std::min((R.n + 255) / 256, ctx->cus * 4);
  const double2* tq = R.tq() + size_t(i) * R.m * R.m;
  const double2* cl = R.c(step) + size_t(i) * R.nq;
  if (precision == GCQ_C128)
    hipLaunchKernelGGL(gcq_columns<double>, dim3(grid), dim3(256), 0, st, q_cur, R.m, R.np, R.nq, R.n,
                       R.ce(step), tq, cl, R.d_x.as<double2>(), R.d_X.as<cpx<double>>());
  else
    hipLaunchKernelGGL(gcq_columns<float>, dim3(grid), dim3(256), 0, st, q_cur, R.m, R.np, R.nq, R.n,
                       R.ce(step), tq, cl, R.d_x.as<double2>(), R.d_X.as<cpx<float>>());
  GCQ_HIP(hipGetLastError());
  GCQ_TRY(gcq_compressed_matvec(ctx, GCQ_PER_FREQUENCY, precision, R.d_X.p, R.d_Y.p, R.L));
  if (precision == GCQ_C128)
    hipLaunchKernelGGL(sum_columns_real<double>, dim3(g2), dim3(256), 0, st, R.d_Y.as<cpx<double>>(), R.L, R.n,
                       out);
  else
    hipLaunchKernelGGL(sum_columns_real<float>, dim3(g2), dim3(256), 0, st, R.d_Y.as<cpx<float>>(), R.L, R.n,
                       out);
  GCQ_HIP(hipGetLastError());
  return GCQ_OK;
}

// the state update into step `step` from the stage values q_prev of step - 1
static int advance_state(gcq_context* ctx, GcqRun& R, int step, const double* q_prev) {
  const int grid = int(std::min<int64_t>((int64_t(R.nq) * R.n + 255) / 256, int64_t(ctx->cus) * 16));
  hipLaunchKernelGGL(gcq_state, dim3(grid), dim3(256), 0, ctx->stream, q_prev, R.m, R.nq, R.n, R.r(step),
                     R.g(step), R.d_x.as<double2>());
  GCQ_HIP(hipGetLastError());
  return GCQ_OK;
}

}  // namespace gcq

using namespace gcq;

extern "C" GCQ_API int gcq_contour_steps(const double* A, int32_t m, double dt_min, double dt_max,
                                         double* args) {
  if (!A || !args) return fail(GCQ_ERR_ARG, "A and args must not be NULL");
  if (m < 1 || m > GCQ_MAX_STAGES) return fail(GCQ_ERR_ARG, "m must be in 1..%d", GCQ_MAX_STAGES);
  if (!(dt_min > 0.0) || !(dt_max >= dt_min) || !std::isfinite(dt_max))
    return fail(GCQ_ERR_ARG, "need 0 < dt_min <= dt_max");
  for (int i = 0; i < m * m; ++i)
    if (!std::isfinite(A[i])) return fail(GCQ_ERR_ARG, "A holds a non-finite entry");
  if (m == 1) {
    if (!(A[0] > 0.0)) return fail(GCQ_ERR_ARG, "a one-stage method needs A > 0");
    args[0] = dt_min * A[0];
    args[1] = dt_max * A[0];
    args[2] = 1.0;
    return GCQ_OK;
  }
  // |lambda(A)|
  std::vector<double> Ar(A, A + m * m);
  std::vector<zd> lam, P, Pinv;
  if (!eigen_small(Ar, m, lam, P, Pinv)) return fail(GCQ_ERR_NUMERIC, "A is not diagonalisable");
  double lmin = 1e300, lmax = 0.0;
  for (const zd& l : lam) {
    lmin = std::min(lmin, std::abs(l));
    lmax = std::max(lmax, std::abs(l));
  }
  if (!(lmin > 0.0)) return fail(GCQ_ERR_ARG, "A is singular");
  // x*: end of the interval (0, x*) where |R(x)| = |e_m^T (I - x A)^{-1} 1| > 1;
  // the last grid point with |R| > 1 on (0, 200], then bisection
  auto growth = [&](double x) {
    std::vector<zd> M(m * m), u(m, 1.0);
    for (int i = 0; i < m; ++i)
      for (int j = 0; j < m; ++j) M[i * m + j] = (i == j ? 1.0 : 0.0) - x * A[i * m + j];
    if (!zsolve(M, u, m, 1)) return 1e300;   // a pole: unbounded growth
    return std::abs(u[m - 1]) - 1.0;
  };
  const int ngrid = 20000;
  const double h = 200.0 / ngrid;
  int last = -1;
  for (int g = 1; g <= ngrid; ++g)
    if (growth(g * h) > 0.0) last = g;
  if (last < 0) return fail(GCQ_ERR_ARG, "the stability function does not exceed 1 on (0, 200]");
  if (last == ngrid) return fail(GCQ_ERR_ARG, "the stability function exceeds 1 beyond x = 200");
  double lo = last * h, hi = (last + 1) * h;
  for (int it = 0; it < 100 && hi - lo > 1e-15 * hi; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (growth(mid) > 0.0) lo = mid; else hi = mid;
  }
  const double xs = 0.5 * (lo + hi);
  args[0] = dt_min / xs;
  args[1] = dt_max / xs;
  args[2] = 5.0 * lmax / lmin;
  return GCQ_OK;
}

extern "C" GCQ_API int gcq_gcq_convolve(gcq_context* ctx, const double* A, int32_t m, const double* dt,
                                        int32_t n_steps, int32_t n_step_points, const gcq_c128* w,
                                        int32_t precision, const double* Q, double* F) {
  const auto t0 = std::chrono::steady_clock::now();
  GcqRun R;
  GCQ_TRY(gcq_prepare(ctx, A, m, dt, n_steps, n_step_points, w, precision, R));
  GCQ_TRY(check_device_ptr(ctx, Q, "Q"));
  GCQ_TRY(check_device_ptr(ctx, F, "F"));
  const int64_t stride = int64_t(m) * R.n;   // one step: m stages of n values
  for (int step = 0; step < n_steps; ++step) {
    if (step > 0) GCQ_TRY(advance_state(ctx, R, step, Q + (step - 1) * stride));
    for (int i = 0; i < m; ++i)
      GCQ_TRY(stage_product(ctx, R, precision, step, Q + step * stride, i, F + step * stride + int64_t(i) * R.n));
  }
  GCQ_HIP(hipStreamSynchronize(ctx->stream));
  ctx->kernel_ms["gcq_convolve"] =
      std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  return GCQ_OK;
}

extern "C" GCQ_API int gcq_gcq_solve(gcq_context* ctx, const double* A, int32_t m, const double* dt,
                                     int32_t n_steps, int32_t n_step_points, const gcq_c128* w,
                                     int32_t precision, const double* F, double* Q, double rtol,
                                     int32_t max_iter, int32_t restart, int32_t* iters_max) {
  const auto t0 = std::chrono::steady_clock::now();
  GcqRun R;
  GCQ_TRY(gcq_prepare(ctx, A, m, dt, n_steps, n_step_points, w, precision, R));
  GCQ_TRY(check_device_ptr(ctx, F, "F"));
  GCQ_TRY(check_device_ptr(ctx, Q, "Q"));
  const int n = R.n, L = R.L;
  const int64_t stride = int64_t(m) * n;
  hipStream_t st = ctx->stream;
  DevBuf d_h, d_B, d_S;
  GCQ_TRY(d_h.ensure(sizeof(double) * size_t(stride)));
  GCQ_HIP(hipMemsetAsync(d_h.p, 0, sizeof(double) * size_t(stride), st));
  GCQ_TRY(d_B.ensure(sizeof(cpx<double>) * size_t(L) * n));
  GCQ_TRY(d_S.ensure(sizeof(cpx<double>) * size_t(L) * n));
  const int grid = int(std::min<int64_t>((int64_t(L) * n + 255) / 256, int64_t(ctx->cus) * 16));
  const int g3 = int(std::min<int64_t>((stride + 255) / 256, int64_t(ctx->cus) * 16));
  int itmax = 0;
  bool missed = false;   // some step's GMRES ended above rtol
  for (int step = 0; step < n_steps; ++step) {
    // history of the earlier steps per stage: the contour sum, no step-point column
    if (step > 0) {
      GCQ_TRY(advance_state(ctx, R, step, Q + (step - 1) * stride));
      for (int i = 0; i < m; ++i)
        GCQ_TRY(stage_product(ctx, R, precision, step, nullptr, i, d_h.as<double>() + int64_t(i) * n));
    }
    // V((dt A)^{-1}) q_n = f_n - h decouples: V(lam_e / dt) y_e = (P^{-1} (f_n - h))_e, q_n = P y
    hipLaunchKernelGGL(gcq_rhs, dim3(grid), dim3(256), 0, st, F + step * stride, d_h.as<double>(), m, R.np, L, n,
                       R.ce(step), R.pinv(), d_B.as<cpx<double>>());
    GCQ_HIP(hipGetLastError());
    gcq_solve_stats ss;
    const int rs = gcq_solve(ctx, d_B.p, d_S.p, rtol, max_iter, restart, precision, &ss);
    if (rs < 0) return rs;
    if (rs == GCQ_NOT_CONVERGED || ss.n_converged < ss.n_systems) missed = true;
    itmax = std::max(itmax, int(ss.iters_max));
    hipLaunchKernelGGL(gcq_take, dim3(g3), dim3(256), 0, st, d_S.as<cpx<double>>(), m, n, R.ke(step), R.P(),
                       Q + step * stride);
    GCQ_HIP(hipGetLastError());
  }
  GCQ_HIP(hipStreamSynchronize(st));
  ctx->kernel_ms["gcq_solve"] =
      std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  if (iters_max) *iters_max = itmax;
  return missed ? GCQ_NOT_CONVERGED : GCQ_OK;
}
