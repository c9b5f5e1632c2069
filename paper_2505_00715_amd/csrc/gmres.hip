// Batched restarted GMRES over all frequencies at once: V(s_k) x_k = b_k, the
// operator being the 3D-ACA compressed product.  Krylov bases, inner products
// and classical Gram-Schmidt (applied twice) in float64; the small Hessenberg
// least-squares problems (Givens rotations, back substitution) on the host.
#include <algorithm>
#include <cmath>
#include <complex>
#include <cstring>

#include "internal.h"
#include "matvec.h"

namespace gcq {

using zc = cpx<double>;

// h[c * L + k] = sum_p conj(V_c[k][p]) w[k][p]  for c < nc;  one block per (c, k)
__global__ void __launch_bounds__(256) gm_dots(const zc* __restrict__ V, const zc* __restrict__ w,
                                               int nc, int L, int n, zc* __restrict__ h) {
  __shared__ double sr[8], si[8];
  const int c = blockIdx.x / L, k = blockIdx.x % L;
  if (c >= nc) return;
  const zc* v = V + (int64_t(c) * L + k) * n;
  const zc* x = w + int64_t(k) * n;
  double ar = 0, ai = 0;
  for (int p = threadIdx.x; p < n; p += blockDim.x) {
    zc a = v[p], b = x[p];
    ar += a.re * b.re + a.im * b.im;
    ai += a.re * b.im - a.im * b.re;
  }
  ar = wave_sum(ar);
  ai = wave_sum(ai);
  const int wv = threadIdx.x / WAVE;
  if ((threadIdx.x & (WAVE - 1)) == 0) { sr[wv] = ar; si[wv] = ai; }
  __syncthreads();
  if (threadIdx.x == 0) {
    double tr = 0, ti = 0;
    for (int q = 0; q < int(blockDim.x / WAVE); ++q) { tr += sr[q]; ti += si[q]; }
    h[int64_t(c) * L + k] = {tr, ti};
  }
}

// w[k][p] -= sum_{c < nc} V_c[k][p] h[c * L + k]
__global__ void gm_sub(const zc* __restrict__ V, zc* __restrict__ w, const zc* __restrict__ h,
                       int nc, int L, int n) {
  const int64_t total = int64_t(L) * n;
  for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < total;
       e += int64_t(gridDim.x) * blockDim.x) {
    const int k = int(e / n);
    zc acc = w[e];
    for (int c = 0; c < nc; ++c) {
      zc p = cmul(V[int64_t(c) * total + e], h[int64_t(c) * L + k]);
      acc.re -= p.re;
      acc.im -= p.im;
    }
    w[e] = acc;
  }
}

// x[k][p] += sum_{c < nc} V_c[k][p] y[c * L + k]
__global__ void gm_update(const zc* __restrict__ V, zc* __restrict__ x, const zc* __restrict__ y,
                          int nc, int L, int n) {
  const int64_t total = int64_t(L) * n;
  for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < total;
       e += int64_t(gridDim.x) * blockDim.x) {
    const int k = int(e / n);
    zc acc = x[e];
    for (int c = 0; c < nc; ++c) {
      zc p = cmul(V[int64_t(c) * total + e], y[int64_t(c) * L + k]);
      acc.re += p.re;
      acc.im += p.im;
    }
    x[e] = acc;
  }
}

// out[k][p] = a[k][p] * s[k]  (s real)
__global__ void gm_scale(const zc* __restrict__ a, zc* __restrict__ out,
                         const double* __restrict__ s, int L, int n) {
  const int64_t total = int64_t(L) * n;
  for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < total;
       e += int64_t(gridDim.x) * blockDim.x) {
    const double f = s[e / n];
    out[e] = {a[e].re * f, a[e].im * f};
  }
}

// r = b - ax
__global__ void gm_resid(const zc* __restrict__ b, const zc* __restrict__ ax, zc* __restrict__ r,
                         int64_t total) {
  for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < total;
       e += int64_t(gridDim.x) * blockDim.x)
    r[e] = {b[e].re - ax[e].re, b[e].im - ax[e].im};
}

__global__ void gm_zero(zc* p, int64_t total) {
  for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < total;
       e += int64_t(gridDim.x) * blockDim.x)
    p[e] = {0.0, 0.0};
}

__global__ void gm_to32(const zc* __restrict__ a, cpx<float>* __restrict__ o, int64_t total) {
  for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < total;
       e += int64_t(gridDim.x) * blockDim.x)
    o[e] = {float(a[e].re), float(a[e].im)};
}

__global__ void gm_from32(const cpx<float>* __restrict__ a, zc* __restrict__ o, int64_t total) {
  for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < total;
       e += int64_t(gridDim.x) * blockDim.x)
    o[e] = {double(a[e].re), double(a[e].im)};
}

// |a_k|^2 per column: one block per column
__global__ void __launch_bounds__(256) gm_norm2(const zc* __restrict__ a, int n,
                                                double* __restrict__ out) {
  __shared__ double sr[8];
  const zc* v = a + int64_t(blockIdx.x) * n;
  double s = 0;
  for (int p = threadIdx.x; p < n; p += blockDim.x) s += v[p].re * v[p].re + v[p].im * v[p].im;
  s = wave_sum(s);
  if ((threadIdx.x & (WAVE - 1)) == 0) sr[threadIdx.x / WAVE] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0;
    for (int q = 0; q < int(blockDim.x / WAVE); ++q) t += sr[q];
    out[blockIdx.x] = t;
  }
}

struct Solver {
  gcq_context* ctx;
  int precision, n, L;
  int64_t total;
  zc* w;            // L x n
  cpx<float>* t32;  // 2 x L x n (product in complex64)
  double* nrm;      // L
  zc* h;            // (restart + 1) x L
  // y = A x  (x, y: L x n complex128, caller order)
  int apply(const zc* x, zc* y) {
    hipStream_t st = ctx->stream;
    if (precision == GCQ_C128) return run_compressed(ctx, GCQ_PER_FREQUENCY, GCQ_C128, x, y);
    hipLaunchKernelGGL(gm_to32, dim3(2048), dim3(256), 0, st, x, t32, total);
    GCQ_TRY(run_compressed(ctx, GCQ_PER_FREQUENCY, precision, t32, t32 + total));
    hipLaunchKernelGGL(gm_from32, dim3(2048), dim3(256), 0, st, t32 + total, y, total);
    return GCQ_OK;
  }
  int norms(const zc* a, std::vector<double>& out) {
    hipLaunchKernelGGL(gm_norm2, dim3(L), dim3(256), 0, ctx->stream, a, n, nrm);
    out.resize(L);
    GCQ_HIP(hipMemcpyAsync(out.data(), nrm, sizeof(double) * L, hipMemcpyDeviceToHost, ctx->stream));
    GCQ_HIP(hipStreamSynchronize(ctx->stream));
    for (auto& v : out) v = std::sqrt(v);
    return GCQ_OK;
  }
};

}  // namespace gcq

using namespace gcq;

extern "C" GCQ_API int gcq_solve(gcq_context* ctx, const void* B_dev, void* X_dev, double rtol,
                                 int32_t max_iter, int32_t restart, int32_t precision,
                                 gcq_solve_stats* stats) {
  if (!ctx) return fail(GCQ_ERR_ARG, "ctx is NULL");
  GCQ_NEED_DEVICE(ctx);
  if (!ctx->F.valid) return fail(GCQ_ERR_STATE, "run gcq_aca3d first");
  if (ctx->F.near_only) return fail(GCQ_ERR_STATE, "the 3D operator holds only the near field of the FMM-based variant: use gcq_fmm3d_matvec");
  if (storage_precision(precision) != ctx->F.precision)
    return fail(GCQ_ERR_ARG, "precision differs from the one the 3D-ACA was built in");
  if (!(rtol > 0.0) || restart < 1 || restart > 200 || max_iter < 0)
    return fail(GCQ_ERR_ARG, "bad solver parameters");
  GCQ_HIP(hipSetDevice(ctx->device));
  GCQ_TRY(check_device_ptr(ctx, B_dev, "B_dev"));
  GCQ_TRY(check_device_ptr(ctx, X_dev, "X_dev"));
  hipStream_t st = ctx->stream;
  const int n = ctx->n, L = ctx->L, m = restart;
  const int64_t total = int64_t(n) * L;
  DevBuf basis, work;
  GCQ_TRY(basis.ensure(size_t(m + 1) * total * sizeof(zc)));
  const size_t wbytes = total * sizeof(zc) + 2 * total * sizeof(cpx<float>) + L * sizeof(double) +
                        size_t(m + 1) * L * sizeof(zc) + 1024;
  GCQ_TRY(work.ensure(wbytes));
  Solver S;
  S.ctx = ctx;
  S.precision = precision;
  S.n = n;
  S.L = L;
  S.total = total;
  S.w = work.as<zc>();
  S.t32 = reinterpret_cast<cpx<float>*>(S.w + total);
  S.nrm = reinterpret_cast<double*>(S.t32 + 2 * total);
  S.h = reinterpret_cast<zc*>(S.nrm + L + 8);
  zc* V = basis.as<zc>();
  const zc* b = reinterpret_cast<const zc*>(B_dev);
  zc* x = reinterpret_cast<zc*>(X_dev);
  const dim3 G(2048), Bk(256);
  hipEvent_t e0, e1;
  GCQ_HIP(hipEventCreate(&e0));
  GCQ_HIP(hipEventCreate(&e1));
  GCQ_HIP(hipEventRecord(e0, st));
  hipLaunchKernelGGL(gm_zero, G, Bk, 0, st, x, total);
  std::vector<double> bn;
  GCQ_TRY(S.norms(b, bn));
  std::vector<int> iters(L, 0), done(L, 0);
  std::vector<double> resid(L, 0.0);
  std::vector<std::complex<double>> H(size_t(L) * (m + 1) * m), g(size_t(L) * (m + 1)), sn(size_t(L) * m);
  std::vector<double> cs(size_t(L) * m);
  std::vector<zc> hbuf(size_t(m + 1) * L), ybuf(size_t(m) * L);
  std::vector<double> scale(L);
  DevBuf dscale;
  GCQ_TRY(dscale.ensure(sizeof(double) * L + sizeof(zc) * size_t(m) * L));
  double* d_scale = dscale.as<double>();
  zc* d_y = reinterpret_cast<zc*>(d_scale + L);
  int total_iters = 0;
  while (true) {
    // r = b - A x into V_0
    GCQ_TRY(S.apply(x, S.w));
    hipLaunchKernelGGL(gm_resid, G, Bk, 0, st, b, S.w, V, total);
    std::vector<double> beta;
    GCQ_TRY(S.norms(V, beta));
    bool all = true;
    for (int k = 0; k < L; ++k) {
      resid[k] = bn[k] > 0 ? beta[k] / bn[k] : 0.0;
      done[k] = bn[k] == 0.0 || beta[k] <= rtol * bn[k];
      all = all && done[k];
    }
    if (all || total_iters >= max_iter) break;
    for (int k = 0; k < L; ++k) scale[k] = beta[k] > 0 ? 1.0 / beta[k] : 0.0;
    GCQ_HIP(hipMemcpyAsync(d_scale, scale.data(), sizeof(double) * L, hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(gm_scale, G, Bk, 0, st, V, V, d_scale, L, n);
    std::fill(H.begin(), H.end(), 0.0);
    std::fill(g.begin(), g.end(), 0.0);
    for (int k = 0; k < L; ++k) g[size_t(k) * (m + 1)] = beta[k];
    int jdone = 0;
    for (int j = 0; j < m; ++j) {
      zc* vj = V + int64_t(j) * total;
      GCQ_TRY(S.apply(vj, S.w));
      // classical Gram-Schmidt, twice
      hipLaunchKernelGGL(gm_dots, dim3((j + 1) * L), Bk, 0, st, V, S.w, j + 1, L, n, S.h);
      GCQ_HIP(hipMemcpyAsync(hbuf.data(), S.h, sizeof(zc) * (j + 1) * L, hipMemcpyDeviceToHost, st));
      hipLaunchKernelGGL(gm_sub, G, Bk, 0, st, V, S.w, S.h, j + 1, L, n);
      hipLaunchKernelGGL(gm_dots, dim3((j + 1) * L), Bk, 0, st, V, S.w, j + 1, L, n, S.h);
      std::vector<zc> h2(size_t(j + 1) * L);
      GCQ_HIP(hipMemcpyAsync(h2.data(), S.h, sizeof(zc) * (j + 1) * L, hipMemcpyDeviceToHost, st));
      hipLaunchKernelGGL(gm_sub, G, Bk, 0, st, V, S.w, S.h, j + 1, L, n);
      std::vector<double> hn;
      GCQ_TRY(S.norms(S.w, hn));
      for (int k = 0; k < L; ++k) scale[k] = hn[k] > 0 ? 1.0 / hn[k] : 0.0;
      GCQ_HIP(hipMemcpyAsync(d_scale, scale.data(), sizeof(double) * L, hipMemcpyHostToDevice, st));
      hipLaunchKernelGGL(gm_scale, G, Bk, 0, st, S.w, V + int64_t(j + 1) * total, d_scale, L, n);
      ++total_iters;
      bool conv_all = true;
      for (int k = 0; k < L; ++k) {
        std::complex<double>* Hk = &H[size_t(k) * (m + 1) * m];
        auto Hat = [&](int r, int c) -> std::complex<double>& { return Hk[size_t(r) * m + c]; };
        for (int c = 0; c <= j; ++c) {
          const zc a = hbuf[size_t(c) * L + k], bb = h2[size_t(c) * L + k];
          Hat(c, j) = {a.re + bb.re, a.im + bb.im};
        }
        Hat(j + 1, j) = hn[k];
        double* csk = &cs[size_t(k) * m];
        std::complex<double>* snk = &sn[size_t(k) * m];
        std::complex<double>* gk = &g[size_t(k) * (m + 1)];
        for (int i = 0; i < j; ++i) {
          std::complex<double> t = csk[i] * Hat(i, j) + snk[i] * Hat(i + 1, j);
          Hat(i + 1, j) = -std::conj(snk[i]) * Hat(i, j) + csk[i] * Hat(i + 1, j);
          Hat(i, j) = t;
        }
        std::complex<double> a = Hat(j, j), bb = Hat(j + 1, j);
        double den = std::sqrt(std::norm(a) + std::norm(bb));
        if (den == 0.0) {
          csk[j] = 1.0;
          snk[j] = 0.0;
        } else if (std::abs(a) == 0.0) {
          csk[j] = 0.0;
          snk[j] = std::conj(bb) / std::abs(bb);
        } else {
          csk[j] = std::abs(a) / den;
          snk[j] = (a / std::abs(a)) * std::conj(bb) / den;
        }
        Hat(j, j) = csk[j] * a + snk[j] * bb;
        Hat(j + 1, j) = 0.0;
        gk[j + 1] = -std::conj(snk[j]) * gk[j];
        gk[j] = csk[j] * gk[j];
        if (!done[k]) {
          iters[k] += 1;
          if (std::abs(gk[j + 1]) <= rtol * bn[k] || hn[k] == 0.0) done[k] = 2;
        }
        conv_all = conv_all && done[k];
      }
      jdone = j + 1;
      if (conv_all || total_iters >= max_iter) break;
    }
    // back substitution per column, then x += V y
    for (int k = 0; k < L; ++k) {
      std::complex<double>* Hk = &H[size_t(k) * (m + 1) * m];
      std::complex<double>* gk = &g[size_t(k) * (m + 1)];
      std::vector<std::complex<double>> y(jdone, 0.0);
      const bool active = beta[k] > 0 && !(bn[k] == 0.0);
      for (int i = jdone - 1; i >= 0 && active; --i) {
        std::complex<double> acc = gk[i];
        for (int c = i + 1; c < jdone; ++c) acc -= Hk[size_t(i) * m + c] * y[c];
        std::complex<double> d = Hk[size_t(i) * m + i];
        y[i] = std::abs(d) > 0 ? acc / d : 0.0;
      }
      for (int c = 0; c < jdone; ++c) ybuf[size_t(c) * L + k] = {y[c].real(), y[c].imag()};
    }
    GCQ_HIP(hipMemcpyAsync(d_y, ybuf.data(), sizeof(zc) * size_t(jdone) * L, hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(gm_update, G, Bk, 0, st, V, x, d_y, jdone, L, n);
    GCQ_HIP(hipGetLastError());
  }
  float msf = 0.f;
  GCQ_HIP(hipEventRecord(e1, st));
  GCQ_HIP(hipEventSynchronize(e1));
  GCQ_HIP(hipEventElapsedTime(&msf, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  const double ms = msf;
  ctx->kernel_ms["solve"] = ms;
  int nconv = 0, imax = 0;
  double rmax = 0;
  for (int k = 0; k < L; ++k) {
    nconv += bn[k] == 0.0 || resid[k] <= rtol;
    imax = std::max(imax, iters[k]);
    rmax = std::max(rmax, resid[k]);
  }
  if (stats) {
    std::memset(stats, 0, sizeof(*stats));
    stats->n_systems = L;
    stats->n_converged = nconv;
    stats->iters_max = imax;
    stats->resid_max = rmax;
    stats->device_ms = ms;
  }
  return nconv == L ? GCQ_OK : GCQ_NOT_CONVERGED;
}
