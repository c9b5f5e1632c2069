// Products with the frequency-dependent operator: permutation in and out of the
// cluster order (with the conjugate-partner rule), and the per-frequency
// H-matrix product (no frequency compression).
#include <algorithm>
#include <cstring>

#include "internal.h"
#include "matvec.h"

namespace gcq {

// Xp[k][p] = X[k][perm[p]] (conjugated when column k is applied through its
// conjugate partner); T_in is the caller's type, T_out the internal one.
template <typename TI, typename TO>
__global__ void permute_in(const cpx<TI>* __restrict__ X, cpx<TO>* __restrict__ Xp,
                           const int* __restrict__ perm, const int* __restrict__ conjflag, int n,
                           int L) {
  const int64_t total = int64_t(n) * L;
  for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < total;
       e += int64_t(gridDim.x) * blockDim.x) {
    const int k = int(e / n), p = int(e % n);
    cpx<TI> v = X[int64_t(k) * n + perm[p]];
    Xp[e] = {TO(v.re), conjflag[k] ? TO(-v.im) : TO(v.im)};
  }
}

template <typename TI, typename TO>
__global__ void permute_out(const cpx<TI>* __restrict__ Yp, cpx<TO>* __restrict__ Y,
                            const int* __restrict__ perm, const int* __restrict__ conjflag, int n,
                            int L) {
  const int64_t total = int64_t(n) * L;
  for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < total;
       e += int64_t(gridDim.x) * blockDim.x) {
    const int k = int(e / n), p = int(e % n);
    cpx<TI> v = Yp[e];
    Y[int64_t(k) * n + perm[p]] = {TO(v.re), conjflag[k] ? TO(-v.im) : TO(v.im)};
  }
}

template <typename T>
__global__ void zero_cpx(cpx<T>* p, int64_t n) {
  for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < n;
       e += int64_t(gridDim.x) * blockDim.x)
    p[e] = {T(0), T(0)};
}

// per-frequency H-matrix product: one wave per (block, column); far blocks as
// U (V^H x), near blocks dense; accumulation into Yp with atomics
template <typename T>
__global__ void __launch_bounds__(64) plainh_kernel(const int* __restrict__ blk, int nblocks,
                                                    const int* __restrict__ far_pos,
                                                    const int* __restrict__ near_pos, int nfar,
                                                    const int* __restrict__ colslot, int L, int n,
                                                    const int64_t* __restrict__ far_off,
                                                    const int* __restrict__ far_rank,
                                                    const cpx<T>* __restrict__ pool,
                                                    const int64_t* __restrict__ near_off,
                                                    int64_t near_slot, const cpx<T>* __restrict__ near,
                                                    const cpx<T>* __restrict__ Xp, cpx<T>* __restrict__ Yp) {
  __shared__ cpx<T> tbuf[64];
  const int lane = threadIdx.x;
  const int64_t total = int64_t(nblocks) * L;
  for (int64_t w = blockIdx.x; w < total; w += gridDim.x) {
    const int b = int(w % nblocks), k = int(w / nblocks);
    const int rb = blk[5 * b], re = blk[5 * b + 1], cb = blk[5 * b + 2], ce = blk[5 * b + 3];
    const int m = re - rb, nn = ce - cb;
    const int slot = colslot[k];
    const cpx<T>* x = Xp + int64_t(k) * n + cb;
    cpx<T>* y = Yp + int64_t(k) * n + rb;
    if (blk[5 * b + 4] & 1) {
      const int f = far_pos[b];
      const int64_t pi = int64_t(slot) * nfar + f;
      const int r = far_rank[pi];
      const cpx<T>* U = pool + far_off[pi];
      const cpx<T>* V = U + int64_t(r) * m;
      __syncthreads();
      for (int c = 0; c < r; ++c) {
        T sr = 0, si = 0;
        for (int j = lane; j < nn; j += WAVE) {
          cpx<T> p = cmulc(V[int64_t(c) * nn + j], x[j]);
          sr += p.re;
          si += p.im;
        }
        sr = wave_sum(sr);
        si = wave_sum(si);
        if (lane == 0) tbuf[c] = {sr, si};
      }
      __syncthreads();
      for (int i = lane; i < m; i += WAVE) {
        cpx<T> acc = {0, 0};
        for (int c = 0; c < r; ++c) {
          cpx<T> p = cmul(U[int64_t(c) * m + i], tbuf[c]);
          acc.re += p.re;
          acc.im += p.im;
        }
        atomicAdd(&y[i].re, acc.re);
        atomicAdd(&y[i].im, acc.im);
      }
    } else {
      const int q = near_pos[b];
      const cpx<T>* D = near + int64_t(slot) * near_slot + near_off[q];
      for (int i = lane; i < m; i += WAVE) {
        cpx<T> acc = {0, 0};
        for (int j = 0; j < nn; ++j) {
          cpx<T> p = cmul(D[int64_t(j) * m + i], x[j]);
          acc.re += p.re;
          acc.im += p.im;
        }
        atomicAdd(&y[i].re, acc.re);
        atomicAdd(&y[i].im, acc.im);
      }
    }
  }
}

template <typename T>
int run_plainh(gcq_context* ctx, const void* X, void* Y, int precision) {
  HFaces& H = ctx->H;
  hipStream_t st = ctx->stream;
  const int n = ctx->n, L = ctx->L;
  const int nb = int(ctx->blocks.size());
  std::vector<int> far_pos(nb, -1), near_pos(nb, -1), colslot(L), conjf(L);
  for (size_t f = 0; f < ctx->far_ids.size(); ++f) far_pos[ctx->far_ids[f]] = int(f);
  for (size_t q = 0; q < ctx->near_ids.size(); ++q) near_pos[ctx->near_ids[q]] = int(q);
  for (int k = 0; k < L; ++k) {
    colslot[k] = H.fslot[ctx->rep[k]];
    conjf[k] = ctx->conj[k];
    if (colslot[k] < 0) return fail(GCQ_ERR_STATE, "frequency %d has no H-matrix", k);
  }
  std::vector<int> meta;
  meta.insert(meta.end(), far_pos.begin(), far_pos.end());
  meta.insert(meta.end(), near_pos.begin(), near_pos.end());
  meta.insert(meta.end(), colslot.begin(), colslot.end());
  meta.insert(meta.end(), conjf.begin(), conjf.end());
  GCQ_TRY(upload(ctx->scratchC, meta, st));
  const int* d_far_pos = ctx->scratchC.as<int>();
  const int* d_near_pos = d_far_pos + nb;
  const int* d_colslot = d_near_pos + nb;
  const int* d_conj = d_colslot + L;
  const int64_t nl = int64_t(n) * L;
  GCQ_TRY(ctx->scratchA.ensure(2 * nl * sizeof(cpx<T>)));
  cpx<T>* Xp = ctx->scratchA.as<cpx<T>>();
  cpx<T>* Yp = Xp + nl;
  const int g = 4096;
  GCQ_TRY(timed_begin(ctx));
  if (precision == GCQ_C128) {
    hipLaunchKernelGGL((permute_in<double, T>), dim3(g), dim3(256), 0, st,
                       (const cpx<double>*)X, Xp, ctx->d_perm.as<int>(), d_conj, n, L);
  } else {
    hipLaunchKernelGGL((permute_in<float, T>), dim3(g), dim3(256), 0, st,
                       (const cpx<float>*)X, Xp, ctx->d_perm.as<int>(), d_conj, n, L);
  }
  hipLaunchKernelGGL(zero_cpx<T>, dim3(g), dim3(256), 0, st, Yp, nl);
  hipLaunchKernelGGL(plainh_kernel<T>, dim3(65536), dim3(64), 0, st, ctx->d_blk.as<int>(), nb,
                     d_far_pos, d_near_pos, int(ctx->far_ids.size()), d_colslot, L, n,
                     H.d_off.as<int64_t>(), H.d_rank.as<int>(), H.factors.as<cpx<T>>(),
                     H.d_near_off.as<int64_t>(), H.near_slot_elems, H.near.as<cpx<T>>(), Xp, Yp);
  if (precision == GCQ_C128) {
    hipLaunchKernelGGL((permute_out<T, double>), dim3(g), dim3(256), 0, st, Yp, (cpx<double>*)Y,
                       ctx->d_perm.as<int>(), d_conj, n, L);
  } else {
    hipLaunchKernelGGL((permute_out<T, float>), dim3(g), dim3(256), 0, st, Yp, (cpx<float>*)Y,
                       ctx->d_perm.as<int>(), d_conj, n, L);
  }
  GCQ_HIP(hipGetLastError());
  timed_end(ctx, "matvec_plainh");
  return GCQ_OK;
}

}  // namespace gcq

using namespace gcq;

extern "C" GCQ_API int gcq_compressed_matvec(gcq_context* ctx, int32_t mode, int32_t precision,
                                             const void* X_dev, void* Y_dev, int32_t n_cols) {
  if (!ctx) return fail(GCQ_ERR_ARG, "ctx is NULL");
  GCQ_NEED_DEVICE(ctx);
  if (precision != GCQ_C128 && precision != GCQ_C64 && precision != GCQ_C64_SPLIT_BF16)
    return fail(GCQ_ERR_ARG, "unknown precision %d", precision);
  if (!ctx->have_tree || !ctx->have_freq) return fail(GCQ_ERR_STATE, "no operator built");
  if (n_cols != ctx->L) return fail(GCQ_ERR_ARG, "n_cols must equal the number of frequencies");
  GCQ_HIP(hipSetDevice(ctx->device));
  GCQ_TRY(check_device_ptr(ctx, X_dev, "X_dev"));
  GCQ_TRY(check_device_ptr(ctx, Y_dev, "Y_dev"));
  if (mode == GCQ_PLAIN_H) {
    if (!ctx->H.valid) return fail(GCQ_ERR_STATE, "run gcq_aca_blocks first");
    if (ctx->H.precision != precision)
      return fail(GCQ_ERR_ARG, "precision differs from the one the H-matrices were built in "
                               "(split-bf16 products apply the 3D-ACA form only)");
    return precision == GCQ_C128 ? run_plainh<double>(ctx, X_dev, Y_dev, precision)
                                 : run_plainh<float>(ctx, X_dev, Y_dev, precision);
  }
  if (mode == GCQ_PER_FREQUENCY || mode == GCQ_WEIGHTED_SUM) {
    if (!ctx->F.valid) return fail(GCQ_ERR_STATE, "run gcq_aca3d first");
    if (ctx->F.near_only) return fail(GCQ_ERR_STATE, "the 3D operator holds only the near field of the FMM-based variant: use gcq_fmm3d_matvec");
    return run_compressed(ctx, mode, precision, X_dev, Y_dev);
  }
  return fail(GCQ_ERR_ARG, "unknown mode %d", mode);
}
