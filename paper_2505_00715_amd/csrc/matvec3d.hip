// Products with the 3D-ACA form (eq. product):
//   PER_FREQUENCY  Y[k] = sum_b sum_d f_{b,d}[k] H_{b,d} X[k][J_b]
//   WEIGHTED_SUM   y    = sum_b sum_d H_{b,d} (sum_k f_{b,d}[k] X[k][J_b])
// with the conjugate-partner rule for columns whose frequency is represented by
// its conjugate.
#include <algorithm>
#include <cstring>

#include "internal.h"
#include "matvec.h"

namespace gcq {

template <typename TI, typename TO>
__global__ void perm_in3(const cpx<TI>* __restrict__ X, cpx<TO>* __restrict__ Xp,
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
__global__ void perm_out3(const cpx<TI>* __restrict__ Yp, cpx<TO>* __restrict__ Y,
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
__global__ void zero3(cpx<T>* p, int64_t n) {
  for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < n;
       e += int64_t(gridDim.x) * blockDim.x)
    p[e] = {T(0), T(0)};
}

// one wave per (block, column): the slices are re-read for every column
template <typename T>
__global__ void __launch_bounds__(64) perfreq_kernel(
    const int* __restrict__ blk, int nblocks, const int* __restrict__ bterm,
    const int* __restrict__ trank, const int64_t* __restrict__ toff,
    const int64_t* __restrict__ tfoff, const cpx<T>* __restrict__ pool,
    const int* __restrict__ colpos, int L, int n, const cpx<T>* __restrict__ Xp,
    cpx<T>* __restrict__ Yp) {
  __shared__ cpx<T> tv[64];
  const int lane = threadIdx.x;
  const int64_t total = int64_t(nblocks) * L;
  for (int64_t w = blockIdx.x; w < total; w += gridDim.x) {
    const int b = int(w % nblocks), k = int(w / nblocks);
    const int rb = blk[5 * b], m = blk[5 * b + 1] - rb, cb = blk[5 * b + 2], nn = blk[5 * b + 3] - cb;
    const int kp = colpos[k];
    const cpx<T>* x = Xp + int64_t(k) * n + cb;
    cpx<T>* y = Yp + int64_t(k) * n + rb;
    for (int d = bterm[b]; d < bterm[b + 1]; ++d) {
      const cpx<T> f = pool[tfoff[d] + kp];
      const int t = trank[d];
      const cpx<T>* S = pool + toff[d];
      if (t < 0) {
        for (int i = lane; i < m; i += WAVE) {
          cpx<T> acc = {0, 0};
          for (int j = 0; j < nn; ++j) {
            cpx<T> p = cmul(S[int64_t(j) * m + i], x[j]);
            acc.re += p.re;
            acc.im += p.im;
          }
          cpx<T> v = cmul(f, acc);
          atomicAdd(&y[i].re, v.re);
          atomicAdd(&y[i].im, v.im);
        }
      } else {
        const cpx<T>* V = S + int64_t(t) * m;
        __syncthreads();
        for (int c = 0; c < t; ++c) {
          T sr = 0, si = 0;
          for (int j = lane; j < nn; j += WAVE) {
            cpx<T> p = cmulc(V[int64_t(c) * nn + j], x[j]);
            sr += p.re;
            si += p.im;
          }
          sr = wave_sum(sr);
          si = wave_sum(si);
          if (lane == 0) tv[c] = cmul(f, cpx<T>{sr, si});
        }
        __syncthreads();
        for (int i = lane; i < m; i += WAVE) {
          cpx<T> acc = {0, 0};
          for (int c = 0; c < t; ++c) {
            cpx<T> p = cmul(S[int64_t(c) * m + i], tv[c]);
            acc.re += p.re;
            acc.im += p.im;
          }
          atomicAdd(&y[i].re, acc.re);
          atomicAdd(&y[i].im, acc.im);
        }
      }
    }
  }
}

// eq. product: one wave per block; per slice the frequency sums w1 (plain
// columns) and w2 (conjugate-represented columns, conjugated input) are formed
// first, then y_I += H w1 + conj(H w2)
template <typename T>
__global__ void __launch_bounds__(64) wsum_kernel(
    const int* __restrict__ blk, int nblocks, const int* __restrict__ bterm,
    const int* __restrict__ trank, const int64_t* __restrict__ toff,
    const int64_t* __restrict__ tfoff, const cpx<T>* __restrict__ pool,
    const int* __restrict__ colpos, const int* __restrict__ conjf, int L, int n,
    const cpx<T>* __restrict__ X, cpx<T>* __restrict__ ybuf, cpx<T>* __restrict__ scratch,
    int64_t sstride) {
  __shared__ cpx<T> t1[64], t2[64];
  const int lane = threadIdx.x;
  cpx<T>* w1 = scratch + int64_t(blockIdx.x) * sstride;
  for (int b = blockIdx.x; b < nblocks; b += gridDim.x) {
    const int rb = blk[5 * b], m = blk[5 * b + 1] - rb, cb = blk[5 * b + 2], nn = blk[5 * b + 3] - cb;
    cpx<T>* w2 = w1 + nn;
    for (int d = bterm[b]; d < bterm[b + 1]; ++d) {
      const cpx<T>* f = pool + tfoff[d];
      __syncthreads();
      for (int j = lane; j < nn; j += WAVE) {
        cpx<T> a1 = {0, 0}, a2 = {0, 0};
        for (int k = 0; k < L; ++k) {
          cpx<T> xv = X[int64_t(k) * n + cb + j];  // X in cluster order, not conjugated
          cpx<T> fk = f[colpos[k]];
          if (conjf[k]) {
            cpx<T> p = cmul(fk, cpx<T>{xv.re, -xv.im});
            a2.re += p.re;
            a2.im += p.im;
          } else {
            cpx<T> p = cmul(fk, xv);
            a1.re += p.re;
            a1.im += p.im;
          }
        }
        w1[j] = a1;
        w2[j] = a2;
      }
      __syncthreads();
      const int t = trank[d];
      const cpx<T>* S = pool + toff[d];
      if (t < 0) {
        for (int i = lane; i < m; i += WAVE) {
          cpx<T> s1 = {0, 0}, s2 = {0, 0};
          for (int j = 0; j < nn; ++j) {
            cpx<T> h = S[int64_t(j) * m + i];
            cpx<T> p1 = cmul(h, w1[j]), p2 = cmul(h, w2[j]);
            s1.re += p1.re; s1.im += p1.im;
            s2.re += p2.re; s2.im += p2.im;
          }
          atomicAdd(&ybuf[rb + i].re, s1.re + s2.re);
          atomicAdd(&ybuf[rb + i].im, s1.im - s2.im);
        }
      } else {
        const cpx<T>* V = S + int64_t(t) * m;
        for (int c = 0; c < t; ++c) {
          T r1 = 0, i1 = 0, r2 = 0, i2 = 0;
          for (int j = lane; j < nn; j += WAVE) {
            cpx<T> v = V[int64_t(c) * nn + j];
            cpx<T> p1 = cmulc(v, w1[j]), p2 = cmulc(v, w2[j]);
            r1 += p1.re; i1 += p1.im;
            r2 += p2.re; i2 += p2.im;
          }
          r1 = wave_sum(r1); i1 = wave_sum(i1);
          r2 = wave_sum(r2); i2 = wave_sum(i2);
          if (lane == 0) { t1[c] = {r1, i1}; t2[c] = {r2, i2}; }
        }
        __syncthreads();
        for (int i = lane; i < m; i += WAVE) {
          cpx<T> s1 = {0, 0}, s2 = {0, 0};
          for (int c = 0; c < t; ++c) {
            cpx<T> u = S[int64_t(c) * m + i];
            cpx<T> p1 = cmul(u, t1[c]), p2 = cmul(u, t2[c]);
            s1.re += p1.re; s1.im += p1.im;
            s2.re += p2.re; s2.im += p2.im;
          }
          atomicAdd(&ybuf[rb + i].re, s1.re + s2.re);
          atomicAdd(&ybuf[rb + i].im, s1.im - s2.im);
        }
      }
    }
  }
}

template <typename T>
static int compressed_impl(gcq_context* ctx, int mode, int precision, const void* X, void* Y) {
  Faces3D& F = ctx->F;
  hipStream_t st = ctx->stream;
  const int n = ctx->n, L = ctx->L, nb = int(ctx->blocks.size());
  std::vector<int> meta(2 * L);
  for (int k = 0; k < L; ++k) {
    meta[k] = ctx->kpos[k];
    meta[L + k] = ctx->conj[k];
  }
  GCQ_TRY(upload(ctx->scratchC, meta, st));
  const int* d_colpos = ctx->scratchC.as<int>();
  const int* d_conj = d_colpos + L;
  const int64_t nl = int64_t(n) * L;
  int maxn = 0;
  for (auto& B : ctx->blocks)
    maxn = std::max(maxn, ctx->clusters[B.col].end - ctx->clusters[B.col].begin);
  const int wgrid = std::min(nb, 4096);
  GCQ_TRY(ctx->scratchB.ensure(size_t(nl + n + 2 * int64_t(maxn) * wgrid) * sizeof(cpx<T>)));
  cpx<T>* Xp = ctx->scratchB.as<cpx<T>>();
  cpx<T>* Yp = Xp + nl;
  const int g = 4096;
  const int* perm = ctx->d_perm.as<int>();
  GCQ_TRY(timed_begin(ctx));
  if (mode == GCQ_PER_FREQUENCY) {
    GCQ_TRY(ctx->scratchA.ensure(size_t(nl) * sizeof(cpx<T>)));
    Yp = ctx->scratchA.as<cpx<T>>();
    if (precision == GCQ_C128)
      hipLaunchKernelGGL((perm_in3<double, T>), dim3(g), dim3(256), 0, st, (const cpx<double>*)X,
                         Xp, perm, d_conj, n, L);
    else
      hipLaunchKernelGGL((perm_in3<float, T>), dim3(g), dim3(256), 0, st, (const cpx<float>*)X, Xp,
                         perm, d_conj, n, L);
    hipLaunchKernelGGL(zero3<T>, dim3(g), dim3(256), 0, st, Yp, nl);
    hipLaunchKernelGGL(perfreq_kernel<T>, dim3(65536), dim3(64), 0, st, ctx->d_blk.as<int>(), nb,
                       F.d_bterm.as<int>(), F.d_trank.as<int>(), F.d_toff.as<int64_t>(),
                       F.d_tfoff.as<int64_t>(), F.slices.as<cpx<T>>(), d_colpos, L, n, Xp, Yp);
    if (precision == GCQ_C128)
      hipLaunchKernelGGL((perm_out3<T, double>), dim3(g), dim3(256), 0, st, Yp, (cpx<double>*)Y,
                         perm, d_conj, n, L);
    else
      hipLaunchKernelGGL((perm_out3<T, float>), dim3(g), dim3(256), 0, st, Yp, (cpx<float>*)Y, perm,
                         d_conj, n, L);
  } else {
    // the weighted sum keeps X unconjugated (the conjugation is applied per slice)
    std::vector<int> zero(L, 0);
    GCQ_TRY(upload(ctx->scratchD, zero, st));
    if (precision == GCQ_C128)
      hipLaunchKernelGGL((perm_in3<double, T>), dim3(g), dim3(256), 0, st, (const cpx<double>*)X,
                         Xp, perm, ctx->scratchD.as<int>(), n, L);
    else
      hipLaunchKernelGGL((perm_in3<float, T>), dim3(g), dim3(256), 0, st, (const cpx<float>*)X, Xp,
                         perm, ctx->scratchD.as<int>(), n, L);
    hipLaunchKernelGGL(zero3<T>, dim3(64), dim3(256), 0, st, Yp, int64_t(n));
    hipLaunchKernelGGL(wsum_kernel<T>, dim3(wgrid), dim3(64), 0, st, ctx->d_blk.as<int>(), nb,
                       F.d_bterm.as<int>(), F.d_trank.as<int>(), F.d_toff.as<int64_t>(),
                       F.d_tfoff.as<int64_t>(), F.slices.as<cpx<T>>(), d_colpos, d_conj, L, n, Xp,
                       Yp, Yp + n, int64_t(2) * maxn);
    if (precision == GCQ_C128)
      hipLaunchKernelGGL((perm_out3<T, double>), dim3(64), dim3(256), 0, st, Yp, (cpx<double>*)Y,
                         perm, ctx->scratchD.as<int>(), n, 1);
    else
      hipLaunchKernelGGL((perm_out3<T, float>), dim3(64), dim3(256), 0, st, Yp, (cpx<float>*)Y,
                         perm, ctx->scratchD.as<int>(), n, 1);
  }
  GCQ_HIP(hipGetLastError());
  timed_end(ctx, mode == GCQ_PER_FREQUENCY ? "matvec_perfreq" : "matvec_wsum");
  return GCQ_OK;
}

int run_compressed(gcq_context* ctx, int mode, int precision, const void* X, void* Y) {
  if (ctx->F.precision != precision)
    return fail(GCQ_ERR_ARG, "precision differs from the one the 3D-ACA was built in");
  return precision == GCQ_C128 ? compressed_impl<double>(ctx, mode, precision, X, Y)
                               : compressed_impl<float>(ctx, mode, precision, X, Y);
}

}  // namespace gcq
