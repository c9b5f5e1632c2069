// Rows of the compressed 3D array at one frequency (gcq_sample_rows):
//   V(s_k)[i, :] = sum_b sum_d f_{b,d}[rep(k)] H_{b,d}[i, :]    (Alg. 1's
// approximant of eq. product), conjugated for a frequency applied through its
// conjugate partner.  Every block whose row cluster holds row i adds its
// columns; the blocks partition the row, so the columns are written, not
// accumulated.
#include <algorithm>
#include <vector>

#include "internal.h"

namespace gcq {

struct RowItem {
  int a;      // output row (position in the caller's list)
  int p;      // internal row position
  int b;      // block whose row cluster holds p
};

// one wave per (row, block): lanes over the block's columns
template <typename T>
__global__ void __launch_bounds__(64) sample_rows_kernel(
    const RowItem* __restrict__ items, int nitems, const int* __restrict__ blk,
    const int* __restrict__ bterm, const int* __restrict__ trank, const int64_t* __restrict__ toff,
    const int64_t* __restrict__ tvoff, const int64_t* __restrict__ tfoff,
    const cpx<T>* __restrict__ pool, const int* __restrict__ perm, int n, int kp, int conj,
    cpx<T>* __restrict__ out) {
  __shared__ cpx<T> urow[64];
  const int lane = threadIdx.x;
  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    const RowItem w = items[it];
    const int rb = blk[5 * w.b], m = blk[5 * w.b + 1] - rb, cb = blk[5 * w.b + 2],
              nn = blk[5 * w.b + 3] - cb;
    const int i = w.p - rb;
    const int d0 = bterm[w.b], d1 = bterm[w.b + 1];
    for (int j0 = 0; j0 < nn; j0 += 64) {
      const int j = j0 + lane;
      cpx<T> acc = {T(0), T(0)};
      for (int d = d0; d < d1; ++d) {
        const cpx<T> f = pool[tfoff[d] + kp];
        const int t = trank[d];
        cpx<T> h = {T(0), T(0)};
        if (t < 0) {   // dense slice, column-major m x nn
          if (j < nn) h = pool[toff[d] + int64_t(j) * m + i];
        } else {       // Ubar (m x t) Vbar^H (t x nn), row i of Ubar staged 64 terms at a time
          for (int c0 = 0; c0 < t; c0 += 64) {
            const int tc = min(64, t - c0);
            __syncthreads();
            if (lane < tc) urow[lane] = pool[toff[d] + int64_t(c0 + lane) * m + i];
            __syncthreads();
            if (j < nn) {
              const cpx<T>* V = pool + tvoff[d] + int64_t(c0) * nn;
              for (int c = 0; c < tc; ++c) {
                const cpx<T> u = urow[c], v = V[int64_t(c) * nn + j];
                h.re += u.re * v.re + u.im * v.im;   // u conj(v)
                h.im += u.im * v.re - u.re * v.im;
              }
            }
          }
        }
        acc.re += f.re * h.re - f.im * h.im;
        acc.im += f.re * h.im + f.im * h.re;
      }
      if (j < nn) out[int64_t(w.a) * n + perm[cb + j]] = {acc.re, conj ? -acc.im : acc.im};
    }
  }
}

}  // namespace gcq

using namespace gcq;

extern "C" GCQ_API int gcq_sample_rows(gcq_context* ctx, const int32_t* rows, int32_t n_rows,
                                       int32_t freq, void* out_dev) {
  if (!ctx) return fail(GCQ_ERR_ARG, "ctx is NULL");
  GCQ_NEED_DEVICE(ctx);
  if (!ctx->F.valid) return fail(GCQ_ERR_STATE, "run gcq_aca3d first");
  if (ctx->F.near_only) return fail(GCQ_ERR_STATE, "the 3D operator holds only the near field of the FMM-based variant: use gcq_fmm3d_matvec");
  if (n_rows < 0) return fail(GCQ_ERR_ARG, "n_rows must be >= 0");
  if (n_rows == 0) return GCQ_OK;
  if (!rows) return fail(GCQ_ERR_ARG, "rows is NULL");
  if (freq < 0 || freq >= ctx->L) return fail(GCQ_ERR_ARG, "frequency %d out of range", freq);
  GCQ_TRY(check_device_ptr(ctx, out_dev, "out_dev"));
  const int n = ctx->n;
  for (int a = 0; a < n_rows; ++a)
    if (rows[a] < 0 || rows[a] >= n) return fail(GCQ_ERR_ARG, "row %d out of range", rows[a]);
  GCQ_HIP(hipSetDevice(ctx->device));
  const Faces3D& F = ctx->F;
  // (row, block) items: the requested positions sorted, each block takes the
  // ones inside its row range
  std::vector<std::pair<int, int>> pos(n_rows);
  for (int a = 0; a < n_rows; ++a) pos[a] = {ctx->iperm[rows[a]], a};
  std::sort(pos.begin(), pos.end());
  std::vector<RowItem> items;
  for (size_t b = 0; b < ctx->blocks.size(); ++b) {
    if (F.brank[b] == 0) continue;
    const Cluster& A = ctx->clusters[ctx->blocks[b].row];
    auto it = std::lower_bound(pos.begin(), pos.end(), std::make_pair(A.begin, -1));
    for (; it != pos.end() && it->first < A.end; ++it) items.push_back({it->second, it->first, int(b)});
  }
  hipStream_t st = ctx->stream;
  const size_t esz = csize(F.precision);
  // rows whose blocks all have rank 0 are zero
  GCQ_HIP(hipMemsetAsync(out_dev, 0, esz * size_t(n_rows) * n, st));
  if (!items.empty()) {
    DevBuf d_items;
    GCQ_TRY(upload(d_items, items, st));
    const int grid = int(std::min<size_t>(items.size(), size_t(ctx->cus) * 64));
    const int kp = ctx->kpos[freq], cj = ctx->conj[freq];
    if (F.precision == GCQ_C128)
      hipLaunchKernelGGL(sample_rows_kernel<double>, dim3(grid), dim3(64), 0, st, d_items.as<RowItem>(),
                         int(items.size()), ctx->d_blk.as<int>(), F.d_bterm.as<int>(), F.d_trank.as<int>(),
                         F.d_toff.as<int64_t>(), F.d_tvoff.as<int64_t>(), F.d_tfoff.as<int64_t>(),
                         F.slices.as<cpx<double>>(), ctx->d_perm.as<int>(), n, kp, cj,
                         reinterpret_cast<cpx<double>*>(out_dev));
    else
      hipLaunchKernelGGL(sample_rows_kernel<float>, dim3(grid), dim3(64), 0, st, d_items.as<RowItem>(),
                         int(items.size()), ctx->d_blk.as<int>(), F.d_bterm.as<int>(), F.d_trank.as<int>(),
                         F.d_toff.as<int64_t>(), F.d_tvoff.as<int64_t>(), F.d_tfoff.as<int64_t>(),
                         F.slices.as<cpx<float>>(), ctx->d_perm.as<int>(), n, kp, cj,
                         reinterpret_cast<cpx<float>*>(out_dev));
    GCQ_HIP(hipGetLastError());
    GCQ_HIP(hipStreamSynchronize(st));   // d_items is freed on return
  }
  return GCQ_OK;
}
