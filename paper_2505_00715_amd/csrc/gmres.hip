// Batched restarted GMRES over all frequencies at once: V(s_k) x_k = b_k, the
// operator being the 3D-ACA compressed product.  Krylov bases, inner products
// and classical Gram-Schmidt (applied twice) in float64.  With graphs enabled
// (the default) one Arnoldi step -- the product, both Gram-Schmidt passes, the
// new basis vector, the Hessenberg column with its Givens rotations and the
// residual estimate of every column -- runs on the device with the step
// index j read from device memory, captured once per solve and replayed; the
// host only reads the number of unconverged columns after each step.  Without
// graphs the small least-squares problems are solved on the host (the
// reference path).
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

// x[k][p] += sum_{c < nc} V_c[k][p] y[c * L + k] (terms with y = 0 skipped:
// the basis vectors of a system beyond the steps its product computed are
// not read)
__global__ void gm_update(const zc* __restrict__ V, zc* __restrict__ x, const zc* __restrict__ y,
                          int nc, int L, int n) {
  const int64_t total = int64_t(L) * n;
  for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < total;
       e += int64_t(gridDim.x) * blockDim.x) {
    const int k = int(e / n);
    zc acc = x[e];
    for (int c = 0; c < nc; ++c) {
      const zc yc = y[int64_t(c) * L + k];
      if (yc.re == 0.0 && yc.im == 0.0) continue;
      zc p = cmul(V[int64_t(c) * total + e], yc);
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

// ---- device-side Arnoldi step (step index j = *dj) ---------------------------------

__global__ void gm_to32_j(const zc* __restrict__ V, const int* __restrict__ dj, cpx<float>* __restrict__ o,
                          int64_t total) {
  const zc* a = V + int64_t(*dj) * total;
  for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < total;
       e += int64_t(gridDim.x) * blockDim.x)
    o[e] = {float(a[e].re), float(a[e].im)};
}

__global__ void gm_copy_j(const zc* __restrict__ V, const int* __restrict__ dj, zc* __restrict__ o, int64_t total) {
  const zc* a = V + int64_t(*dj) * total;
  for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < total;
       e += int64_t(gridDim.x) * blockDim.x)
    o[e] = a[e];
}

// gm_dots over the first *dj + 1 basis vectors (the grid covers the most)
__global__ void __launch_bounds__(256) gm_dots_j(const zc* __restrict__ V, const zc* __restrict__ w,
                                                 const int* __restrict__ dj, int L, int n, zc* __restrict__ h) {
  __shared__ double sr[8], si[8];
  const int nc = *dj + 1;
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

__global__ void gm_sub_j(const zc* __restrict__ V, zc* __restrict__ w, const zc* __restrict__ h,
                         const int* __restrict__ dj, int L, int n) {
  const int nc = *dj + 1;
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

// per column k: the Hessenberg column j (the two Gram-Schmidt passes' sums and
// the new vector's norm), the earlier Givens rotations applied to it, a new
// rotation that zeroes its subdiagonal, the rotated right-hand side g and the
// residual estimate |g[j + 1]|; the scale of the next basis vector; the number
// of unconverged columns into *active.  H: [k][row][col] (m + 1) x m
__global__ void gm_givens(const int* __restrict__ dj, const zc* __restrict__ h1, const zc* __restrict__ h2,
                          const double* __restrict__ nrm, zc* __restrict__ H, double* __restrict__ cs,
                          zc* __restrict__ sn, zc* __restrict__ g, int* __restrict__ done,
                          int* __restrict__ iters, const double* __restrict__ bn, double rtol,
                          double* __restrict__ scale, int* __restrict__ active, int* __restrict__ deep, int m,
                          int L) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= L) return;
  const int j = *dj;
  zc* Hk = H + int64_t(k) * (m + 1) * m;
  double* csk = cs + int64_t(k) * m;
  zc* snk = sn + int64_t(k) * m;
  zc* gk = g + int64_t(k) * (m + 1);
  for (int c = 0; c <= j; ++c) {
    const zc a = h1[int64_t(c) * L + k], b = h2[int64_t(c) * L + k];
    Hk[c * m + j] = {a.re + b.re, a.im + b.im};
  }
  const double hn = sqrt(nrm[k]);
  Hk[(j + 1) * m + j] = {hn, 0.0};
  for (int i = 0; i < j; ++i) {
    const zc hi = Hk[i * m + j], hi1 = Hk[(i + 1) * m + j];
    const zc s = snk[i];
    // t = c h_i + s h_{i+1};  h_{i+1} = -conj(s) h_i + c h_{i+1}
    const zc t = {csk[i] * hi.re + (s.re * hi1.re - s.im * hi1.im), csk[i] * hi.im + (s.re * hi1.im + s.im * hi1.re)};
    const zc u = {-(s.re * hi.re + s.im * hi.im) + csk[i] * hi1.re, -(s.re * hi.im - s.im * hi.re) + csk[i] * hi1.im};
    Hk[(i + 1) * m + j] = u;
    Hk[i * m + j] = t;
  }
  const zc a = Hk[j * m + j], bb = Hk[(j + 1) * m + j];
  const double na = sqrt(a.re * a.re + a.im * a.im), nb = sqrt(bb.re * bb.re + bb.im * bb.im);
  const double den = sqrt(na * na + nb * nb);
  double c;
  zc sv;
  if (den == 0.0) {
    c = 1.0;
    sv = {0.0, 0.0};
  } else if (na == 0.0) {
    c = 0.0;
    sv = {bb.re / nb, -bb.im / nb};
  } else {
    c = na / den;
    // (a / |a|) conj(b) / den
    const zc ph = {a.re / na, a.im / na};
    sv = {(ph.re * bb.re + ph.im * bb.im) / den, (ph.im * bb.re - ph.re * bb.im) / den};
  }
  csk[j] = c;
  snk[j] = sv;
  Hk[j * m + j] = {c * a.re + (sv.re * bb.re - sv.im * bb.im), c * a.im + (sv.re * bb.im + sv.im * bb.re)};
  Hk[(j + 1) * m + j] = {0.0, 0.0};
  const zc gj = gk[j];
  gk[j + 1] = {-(sv.re * gj.re + sv.im * gj.im), -(sv.re * gj.im - sv.im * gj.re)};
  gk[j] = {c * gj.re, c * gj.im};
  int dk = done[k];
  const double r = sqrt(gk[j + 1].re * gk[j + 1].re + gk[j + 1].im * gk[j + 1].im);
  if (!dk) {
    iters[k] += 1;
    if (r <= rtol * bn[k] || hn == 0.0) dk = 2;
    done[k] = dk;
  }
  // below half the tolerance: the system's product may stop (its residual at
  // the restart then stays below the tolerance)
  if (r <= 0.5 * rtol * bn[k] || hn == 0.0) deep[k] = 1;
  scale[k] = hn > 0 ? 1.0 / hn : 0.0;
  if (!dk) atomicAdd(active, 1);
}

__global__ void gm_scale_j(const zc* __restrict__ a, zc* __restrict__ V, const int* __restrict__ dj,
                           const double* __restrict__ s, int L, int n) {
  const int64_t total = int64_t(L) * n;
  zc* out = V + int64_t(*dj + 1) * total;
  for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < total;
       e += int64_t(gridDim.x) * blockDim.x) {
    const double f = s[e / n];
    out[e] = {a[e].re * f, a[e].im * f};
  }
}

// start of step j = *dj: the unconverged count starts at 0; a 32-column
// frequency tile whose systems are all below half the tolerance (deep) is left
// out of this step's product (mask 0), the others record that their basis is
// valid through step j (tvalid: the steps a tile's systems may use in the back
// substitution)
__global__ void gm_begin_step(int* __restrict__ active, const int* __restrict__ dj, const int* __restrict__ deep,
                              int* __restrict__ mask, int* __restrict__ tvalid, int L) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *active = 0;
  const int nkt = (L + 31) / 32, j = *dj;
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < nkt; t += gridDim.x * blockDim.x) {
    int any = 0;
    for (int k = 32 * t; k < min(L, 32 * t + 32); ++k) any |= deep[k] == 0;
    mask[t] = any;
    if (any) tvalid[t] = j + 1;
  }
}

// end of a step: j + 1
__global__ void gm_next_j(int* __restrict__ dj) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *dj += 1;
}

// back substitution per column over its first min(jdone, tvalid of its tile)
// rows (the steps whose basis vectors its product computed): y[c * L + k],
// zero in the rows beyond
__global__ void gm_backsub(const zc* __restrict__ H, const zc* __restrict__ g, const double* __restrict__ beta,
                           const double* __restrict__ bn, const int* __restrict__ tvalid, int jdone, int m, int L,
                           zc* __restrict__ y) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= L) return;
  const zc* Hk = H + int64_t(k) * (m + 1) * m;
  const zc* gk = g + int64_t(k) * (m + 1);
  const bool act = beta[k] > 0 && !(bn[k] == 0.0);
  const int jd = min(jdone, tvalid[k / 32]);
  for (int i = jdone - 1; i >= jd; --i) y[int64_t(i) * L + k] = {0.0, 0.0};
  for (int i = jd - 1; i >= 0; --i) {
    zc acc = act ? gk[i] : zc{0.0, 0.0};
    if (act)
      for (int c = i + 1; c < jd; ++c) {
        const zc p = cmul(Hk[i * m + c], y[int64_t(c) * L + k]);
        acc.re -= p.re;
        acc.im -= p.im;
      }
    const zc d = Hk[i * m + i];
    const double dd = d.re * d.re + d.im * d.im;
    y[int64_t(i) * L + k] = (act && dd > 0) ? zc{(acc.re * d.re + acc.im * d.im) / dd, (acc.im * d.re - acc.re * d.im) / dd}
                                            : zc{0.0, 0.0};
  }
}

__global__ void gm_zero_d(double* p, int64_t cnt) {
  for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < cnt; e += int64_t(gridDim.x) * blockDim.x)
    p[e] = 0.0;
}

// device state of the graph path
struct DevState {
  zc *H = nullptr, *sn = nullptr, *g = nullptr, *h2 = nullptr;
  double *cs = nullptr, *bn = nullptr, *beta = nullptr, *scale = nullptr;
  int *done = nullptr, *iters = nullptr, *dj = nullptr, *active = nullptr;
  int *mask = nullptr, *tvalid = nullptr;   // per 32-column frequency tile
  int* deep = nullptr;                      // per system: residual below half the tolerance
  int* host_active = nullptr;
  hipGraphExec_t exec = nullptr;
};

// one Arnoldi step (reads j = *D.dj) captured into D.exec
static int capture_step(gcq_context* ctx, Solver& S, DevState& D, zc* V, int m, double rtol) {
  Faces3D& F = ctx->F;
  if (!F.graphs.cap) GCQ_HIP(hipStreamCreateWithFlags(&F.graphs.cap, hipStreamNonBlocking));
  hipStream_t cs = F.graphs.cap;
  const int L = S.L, n = S.n;
  const int64_t total = S.total;
  const dim3 G(2048), Bk(256);
  hipGraph_t graph = nullptr;
  GCQ_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
  hipLaunchKernelGGL(gm_begin_step, dim3(1), dim3(64), 0, cs, D.active, D.dj, D.deep, D.mask, D.tvalid, L);
  if (S.precision == GCQ_C128) {
    zc* tmp = reinterpret_cast<zc*>(S.t32);
    hipLaunchKernelGGL(gm_copy_j, G, Bk, 0, cs, V, D.dj, tmp, total);
    enqueue_perfreq_any(ctx, cs, S.precision, tmp, S.w, D.mask);
  } else {
    hipLaunchKernelGGL(gm_to32_j, G, Bk, 0, cs, V, D.dj, S.t32, total);
    enqueue_perfreq_any(ctx, cs, S.precision, S.t32, S.t32 + total, D.mask);
    hipLaunchKernelGGL(gm_from32, G, Bk, 0, cs, S.t32 + total, S.w, total);
  }
  hipLaunchKernelGGL(gm_dots_j, dim3((m + 1) * L), Bk, 0, cs, V, S.w, D.dj, L, n, S.h);
  hipLaunchKernelGGL(gm_sub_j, G, Bk, 0, cs, V, S.w, S.h, D.dj, L, n);
  hipLaunchKernelGGL(gm_dots_j, dim3((m + 1) * L), Bk, 0, cs, V, S.w, D.dj, L, n, D.h2);
  hipLaunchKernelGGL(gm_sub_j, G, Bk, 0, cs, V, S.w, D.h2, D.dj, L, n);
  hipLaunchKernelGGL(gm_norm2, dim3(L), Bk, 0, cs, S.w, n, S.nrm);
  hipLaunchKernelGGL(gm_givens, dim3((L + 255) / 256), Bk, 0, cs, D.dj, S.h, D.h2, S.nrm, D.H, D.cs, D.sn, D.g,
                     D.done, D.iters, D.bn, rtol, D.scale, D.active, D.deep, m, L);
  hipLaunchKernelGGL(gm_scale_j, G, Bk, 0, cs, S.w, V, D.dj, D.scale, L, n);
  hipLaunchKernelGGL(gm_next_j, dim3(1), dim3(64), 0, cs, D.dj);
  const hipError_t ce = hipGetLastError();
  GCQ_HIP(hipStreamEndCapture(cs, &graph));
  if (ce != hipSuccess) {
    (void)hipGraphDestroy(graph);
    return fail(GCQ_ERR_HIP, "capture of the Arnoldi step failed: %s", hipGetErrorString(ce));
  }
  const hipError_t ie = hipGraphInstantiate(&D.exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (ie != hipSuccess) return fail(GCQ_ERR_HIP, "graph instantiation failed: %s", hipGetErrorString(ie));
  return GCQ_OK;
}

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
  std::vector<int> iters(L, 0), done(L, 0), deep(L, 0);
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
  // device-side Arnoldi step, replayed as a graph (tuning product_graph)
  const bool use_graph = ctx->tune.product_graph != 0;
  DevState D;
  DevBuf dstate;
  int* pinned_active = nullptr;
  if (use_graph) {
    GCQ_TRY(prepare_perfreq(ctx, precision));
    const size_t zc_n = size_t(L) * (m + 1) * m + size_t(L) * m + size_t(L) * (m + 1) + size_t(m + 1) * L;
    const int nkt = (L + 31) / 32;
    // fourteen arrays, each rounded up to 256 bytes
    const size_t bytes = zc_n * sizeof(zc) + sizeof(double) * (size_t(L) * m + 2 * L) +
                         sizeof(int) * (3 * L + 2 + 2 * nkt) + 14 * 256;
    GCQ_TRY(dstate.ensure(bytes));
    unsigned char* q = dstate.as<unsigned char>();
    auto take = [&](size_t b) { unsigned char* r = q; q += (b + 255) & ~size_t(255); return r; };
    D.H = reinterpret_cast<zc*>(take(sizeof(zc) * size_t(L) * (m + 1) * m));
    D.sn = reinterpret_cast<zc*>(take(sizeof(zc) * size_t(L) * m));
    D.g = reinterpret_cast<zc*>(take(sizeof(zc) * size_t(L) * (m + 1)));
    D.h2 = reinterpret_cast<zc*>(take(sizeof(zc) * size_t(m + 1) * L));
    D.cs = reinterpret_cast<double*>(take(sizeof(double) * size_t(L) * m));
    D.bn = reinterpret_cast<double*>(take(sizeof(double) * L));
    D.beta = reinterpret_cast<double*>(take(sizeof(double) * L));
    D.done = reinterpret_cast<int*>(take(sizeof(int) * L));
    D.iters = reinterpret_cast<int*>(take(sizeof(int) * L));
    D.dj = reinterpret_cast<int*>(take(sizeof(int)));
    D.active = reinterpret_cast<int*>(take(sizeof(int)));
    D.mask = reinterpret_cast<int*>(take(sizeof(int) * nkt));
    D.tvalid = reinterpret_cast<int*>(take(sizeof(int) * nkt));
    D.deep = reinterpret_cast<int*>(take(sizeof(int) * L));
    D.scale = d_scale;
    GCQ_HIP(hipHostMalloc(reinterpret_cast<void**>(&pinned_active), sizeof(int), hipHostMallocDefault));
    D.host_active = pinned_active;
    GCQ_HIP(hipMemcpyAsync(D.bn, bn.data(), sizeof(double) * L, hipMemcpyHostToDevice, st));
    GCQ_HIP(hipMemsetAsync(D.iters, 0, sizeof(int) * L, st));
  }
  struct Cleanup {
    DevState* d;
    int* pinned;
    ~Cleanup() {
      if (d->exec) (void)hipGraphExecDestroy(d->exec);
      if (pinned) (void)hipHostFree(pinned);
    }
  } cleanup{&D, pinned_active};
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
      deep[k] = bn[k] == 0.0 || beta[k] <= 0.5 * rtol * bn[k];
      all = all && done[k];
    }
    if (all || total_iters >= max_iter) break;
    for (int k = 0; k < L; ++k) scale[k] = beta[k] > 0 ? 1.0 / beta[k] : 0.0;
    GCQ_HIP(hipMemcpyAsync(d_scale, scale.data(), sizeof(double) * L, hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(gm_scale, G, Bk, 0, st, V, V, d_scale, L, n);
    if (use_graph) {
      // per restart: right-hand sides g = beta e_1, Hessenberg zero, flags, j = 0
      std::vector<zc> g0(size_t(L) * (m + 1), zc{0.0, 0.0});
      for (int k = 0; k < L; ++k) g0[size_t(k) * (m + 1)] = {beta[k], 0.0};
      std::vector<int> dn(done.begin(), done.end());
      GCQ_HIP(hipMemcpyAsync(D.g, g0.data(), sizeof(zc) * g0.size(), hipMemcpyHostToDevice, st));
      GCQ_HIP(hipMemcpyAsync(D.done, dn.data(), sizeof(int) * L, hipMemcpyHostToDevice, st));
      GCQ_HIP(hipMemcpyAsync(D.deep, deep.data(), sizeof(int) * L, hipMemcpyHostToDevice, st));
      GCQ_HIP(hipMemcpyAsync(D.beta, beta.data(), sizeof(double) * L, hipMemcpyHostToDevice, st));
      hipLaunchKernelGGL(gm_zero_d, G, Bk, 0, st, reinterpret_cast<double*>(D.H), int64_t(L) * (m + 1) * m * 2);
      GCQ_HIP(hipMemsetAsync(D.dj, 0, sizeof(int), st));
      GCQ_HIP(hipMemsetAsync(D.tvalid, 0, sizeof(int) * ((L + 31) / 32), st));
      if (!D.exec) GCQ_TRY(capture_step(ctx, S, D, V, m, rtol));
      int jdone = 0;
      for (int j = 0; j < m; ++j) {
        GCQ_HIP(hipGraphLaunch(D.exec, st));
        int act = 0;
        GCQ_HIP(hipMemcpyAsync(D.host_active, D.active, sizeof(int), hipMemcpyDeviceToHost, st));
        GCQ_HIP(hipStreamSynchronize(st));
        act = *D.host_active;
        ++total_iters;
        jdone = j + 1;
        if (act == 0 || total_iters >= max_iter) break;
      }
      hipLaunchKernelGGL(gm_backsub, dim3((L + 255) / 256), Bk, 0, st, D.H, D.g, D.beta, D.bn, D.tvalid, jdone, m,
                         L, d_y);
      hipLaunchKernelGGL(gm_update, G, Bk, 0, st, V, x, d_y, jdone, L, n);
      GCQ_HIP(hipGetLastError());
      continue;
    }
    std::fill(H.begin(), H.end(), 0.0);
    std::fill(g.begin(), g.end(), 0.0);
    for (int k = 0; k < L; ++k) g[size_t(k) * (m + 1)] = beta[k];
    int jdone = 0;
    // steps whose basis each 32-column tile may use (as the graph path, whose
    // product leaves out tiles whose systems have all converged)
    std::vector<int> tvalid((L + 31) / 32, 0);
    for (int j = 0; j < m; ++j) {
      for (int t = 0; t < int(tvalid.size()); ++t) {
        bool any = false;
        for (int k = 32 * t; k < std::min(L, 32 * t + 32); ++k) any = any || !deep[k];
        if (any) tvalid[t] = j + 1;
      }
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
        if (std::abs(gk[j + 1]) <= 0.5 * rtol * bn[k] || hn[k] == 0.0) deep[k] = 1;
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
      const int jd = std::min(jdone, tvalid[k / 32]);
      for (int i = jd - 1; i >= 0 && active; --i) {
        std::complex<double> acc = gk[i];
        for (int c = i + 1; c < jd; ++c) acc -= Hk[size_t(i) * m + c] * y[c];
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
  if (use_graph) GCQ_HIP(hipMemcpy(iters.data(), D.iters, sizeof(int) * L, hipMemcpyDeviceToHost));
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
