// Dense entries V(s_f)[rows[a], cols[b]] (single layer) and K(s_f)[rows[a],
// cols[b]] (double layer) for index and frequency lists.
#include "internal.h"

namespace gcq {

// (1 + kappa r) exp(-kappa r) for kappa = sr + i si
__device__ __forceinline__ cpx<float> dlp_radial(float r, float sr, float si) {
  const float e = expf(-sr * r);
  float sn, cs;
  sincosf(si * r, &sn, &cs);
  const float a = 1.f + sr * r, b = si * r;
  return {e * (a * cs + b * sn), e * (b * cs - a * sn)};
}
__device__ __forceinline__ cpx<double> dlp_radial(double r, double sr, double si) {
  const double e = exp(-sr * r);
  double sn, cs;
  sincos(si * r, &sn, &cs);
  const double a = 1.0 + sr * r, b = si * r;
  return {e * (a * cs + b * sn), e * (b * cs - a * sn)};
}

// unit normal of panel p from its vertices, (v1 - v0) x (v2 - v0) / |.|
__device__ __forceinline__ void panel_normal(const Tab& t, int p, double nrm[3]) {
  const int n = t.n;
  double v[9];
#pragma unroll
  for (int c = 0; c < 9; ++c) v[c] = t.vert[c * n + p];
  const double ax = v[3] - v[0], ay = v[4] - v[1], az = v[5] - v[2];
  const double bx = v[6] - v[0], by = v[7] - v[1], bz = v[8] - v[2];
  const double cx = ay * bz - az * by, cy = az * bx - ax * bz, cz = ax * by - ay * bx;
  const double inv = 1.0 / sqrt(cx * cx + cy * cy + cz * cz);
  nrm[0] = cx * inv;
  nrm[1] = cy * inv;
  nrm[2] = cz * inv;
}

// double-layer entry: sum_q w_q (d . n_j) (1 + kappa r) exp(-kappa r) / (4 pi r^3),
// d = x_i - y_q; self 0 (x_i lies in the plane of its flat panel), near tier
// on the 112-point rule in double, far tier on the 7-point rule in T
template <typename T>
__device__ __forceinline__ cpx<T> dlp_entry(const Tab& t, int pi, int pj, double sr, double si) {
  if (pi == pj) return {T(0), T(0)};
  const int n = t.n;
  double nrm[3];
  panel_normal(t, pj, nrm);
  if (is_near(t, pi, pj)) {
    const double xi = t.cen[pi], yi = t.cen[n + pi], zi = t.cen[2 * n + pi];
    double v[9];
#pragma unroll
    for (int c = 0; c < 9; ++c) v[c] = t.vert[c * n + pj];
    const double wa = t.area[pj] * INV4PI;
    double ar = 0.0, ai = 0.0;
    for (int a = 0; a < NQ_NEAR; ++a) {
      const double b0 = t.K->nb[a][0], b1 = t.K->nb[a][1], b2 = t.K->nb[a][2];
      const double dx = xi - (b0 * v[0] + b1 * v[3] + b2 * v[6]);
      const double dy = yi - (b0 * v[1] + b1 * v[4] + b2 * v[7]);
      const double dz = zi - (b0 * v[2] + b1 * v[5] + b2 * v[8]);
      const double r2 = dx * dx + dy * dy + dz * dz, r = sqrt(r2);
      const double f = t.K->nw[a] * wa * (dx * nrm[0] + dy * nrm[1] + dz * nrm[2]) / (r2 * r);
      const cpx<double> g = dlp_radial(r, sr, si);
      ar += f * g.re;
      ai += f * g.im;
    }
    return {T(ar), T(ai)};
  }
  const T* q = FarData<T>::q(t);
  const T* c = FarData<T>::c(t);
  const T xi = c[pi], yi = c[n + pi], zi = c[2 * n + pi];
  const T nx = T(nrm[0]), ny = T(nrm[1]), nz = T(nrm[2]);
  T ar = T(0), ai = T(0);
#pragma unroll
  for (int a = 0; a < NQ_FAR; ++a) {
    const T dx = xi - q[a * n + pj];
    const T dy = yi - q[(7 + a) * n + pj];
    const T dz = zi - q[(14 + a) * n + pj];
    const T w = q[(21 + a) * n + pj];
    const T r2 = dx * dx + dy * dy + dz * dz, r = sqrt(r2);
    const T f = w * (dx * nx + dy * ny + dz * nz) / (r2 * r);
    const cpx<T> g = dlp_radial(r, T(sr), T(si));
    ar += f * g.re;
    ai += f * g.im;
  }
  return {ar, ai};
}

// one thread per (a, b); the frequencies loop inside so that the geometry of
// the pair is loaded once.  out[(f * ncol + b) * nrow + a].
template <typename T, bool DLP>
__global__ void __launch_bounds__(256) assemble_kernel(Tab tab, const int* __restrict__ prow,
                                                       const int* __restrict__ pcol, int64_t nrow,
                                                       int64_t ncol, const double2* __restrict__ sig,
                                                       int nf, cpx<T>* __restrict__ out) {
  const int64_t id = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (id >= nrow * ncol) return;
  const int64_t a = id % nrow, b = id / nrow;
  const int pi = prow[a], pj = pcol[b];
  for (int f = 0; f < nf; ++f) {
    double2 s = sig[f];
    out[(int64_t(f) * ncol + b) * nrow + a] =
        DLP ? dlp_entry<T>(tab, pi, pj, s.x, s.y) : entry<T>(tab, pi, pj, s.x, s.y, false);
  }
}

template <bool DLP>
static int assemble(gcq_context* ctx, const int32_t* rows, int64_t n_rows, const int32_t* cols, int64_t n_cols,
                    const int32_t* freq_idx, int32_t n_fidx, int32_t precision, void* out_dev) {
  if (!ctx) return fail(GCQ_ERR_ARG, "ctx is NULL");
  GCQ_NEED_DEVICE(ctx);
  if (!ctx->have_tree) return fail(GCQ_ERR_STATE, "build the cluster tree first");
  if (!ctx->have_freq) return fail(GCQ_ERR_STATE, "set the frequencies first");
  if (precision != GCQ_C128 && precision != GCQ_C64)
    return fail(GCQ_ERR_ARG, "unknown precision %d", precision);
  if (n_rows < 0 || n_cols < 0 || n_fidx < 0) return fail(GCQ_ERR_ARG, "negative size");
  if (n_rows == 0 || n_cols == 0 || n_fidx == 0) return GCQ_OK;
  if (!rows || !cols || !freq_idx) return fail(GCQ_ERR_ARG, "index list is NULL");
  GCQ_HIP(hipSetDevice(ctx->device));
  GCQ_TRY(check_device_ptr(ctx, out_dev, "out_dev"));
  std::vector<int32_t> pr(n_rows), pc(n_cols);
  for (int64_t a = 0; a < n_rows; ++a) {
    if (rows[a] < 0 || rows[a] >= ctx->n) return fail(GCQ_ERR_ARG, "row index out of range");
    pr[a] = ctx->iperm[rows[a]];
  }
  for (int64_t b = 0; b < n_cols; ++b) {
    if (cols[b] < 0 || cols[b] >= ctx->n) return fail(GCQ_ERR_ARG, "column index out of range");
    pc[b] = ctx->iperm[cols[b]];
  }
  std::vector<double2> sig(n_fidx);
  for (int f = 0; f < n_fidx; ++f) {
    if (freq_idx[f] < 0 || freq_idx[f] >= ctx->L)
      return fail(GCQ_ERR_ARG, "frequency index out of range");
    std::complex<double> sg = ctx->s[freq_idx[f]] / ctx->c;
    sig[f] = make_double2(sg.real(), sg.imag());
  }
  GCQ_TRY(upload(ctx->scratchA, pr, ctx->stream));
  GCQ_TRY(upload(ctx->scratchB, pc, ctx->stream));
  GCQ_TRY(upload(ctx->scratchC, sig, ctx->stream));
  const int64_t total = n_rows * n_cols;
  const int64_t nblk = (total + 255) / 256;
  if (nblk > 0x7fffffff) return fail(GCQ_ERR_ARG, "request too large");
  GCQ_TRY(timed_begin(ctx));
  if (precision == GCQ_C128)
    hipLaunchKernelGGL((assemble_kernel<double, DLP>), dim3(unsigned(nblk)), dim3(256), 0, ctx->stream,
                       ctx->tab(), ctx->scratchA.as<int>(), ctx->scratchB.as<int>(), n_rows, n_cols,
                       ctx->scratchC.as<double2>(), n_fidx, reinterpret_cast<cpx<double>*>(out_dev));
  else
    hipLaunchKernelGGL((assemble_kernel<float, DLP>), dim3(unsigned(nblk)), dim3(256), 0, ctx->stream,
                       ctx->tab(), ctx->scratchA.as<int>(), ctx->scratchB.as<int>(), n_rows, n_cols,
                       ctx->scratchC.as<double2>(), n_fidx, reinterpret_cast<cpx<float>*>(out_dev));
  GCQ_HIP(hipGetLastError());
  timed_end(ctx, DLP ? "assemble_dlp" : "assemble");
  return GCQ_OK;
}

}  // namespace gcq

using namespace gcq;

extern "C" GCQ_API int gcq_assemble_slices(gcq_context* ctx, const int32_t* rows, int64_t n_rows,
                                           const int32_t* cols, int64_t n_cols,
                                           const int32_t* freq_idx, int32_t n_fidx,
                                           int32_t precision, void* out_dev) {
  return assemble<false>(ctx, rows, n_rows, cols, n_cols, freq_idx, n_fidx, precision, out_dev);
}

extern "C" GCQ_API int gcq_assemble_dlp_slices(gcq_context* ctx, const int32_t* rows, int64_t n_rows,
                                               const int32_t* cols, int64_t n_cols,
                                               const int32_t* freq_idx, int32_t n_fidx,
                                               int32_t precision, void* out_dev) {
  return assemble<true>(ctx, rows, n_rows, cols, n_cols, freq_idx, n_fidx, precision, out_dev);
}
