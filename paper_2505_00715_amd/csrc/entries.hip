// Dense entries V(s_f)[rows[a], cols[b]] (single layer) and K(s_f)[rows[a],
// cols[b]] (double layer) for index and frequency lists.
#include "internal.h"

namespace gcq {

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
        DLP ? dlp_entry_part<T>(tab, pi, pj, s.x, s.y, false, 0, 1) : entry<T>(tab, pi, pj, s.x, s.y, false);
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
