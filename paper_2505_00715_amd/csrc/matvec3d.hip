// Products with the 3D-ACA form (eq. product):
//   PER_FREQUENCY  Y[k] = sum_b sum_d f_{b,d}[k] H_{b,d} X[k][J_b]
//   WEIGHTED_SUM   y    = sum_b sum_d H_{b,d} (sum_k f_{b,d}[k] X[k][J_b])
// with the conjugate-partner rule for columns whose frequency is represented by
// its conjugate.
#include <algorithm>
#include <cstring>

#include "internal.h"
#include <type_traits>

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

// Xp[p][k] = X[k][perm[p]] (frequency fastest), conjugated for columns applied
// through their conjugate partner; and the inverse for the result
template <typename TI, typename TO>
__global__ void perm_in_t(const cpx<TI>* __restrict__ X, cpx<TO>* __restrict__ Xp,
                          const int* __restrict__ perm, const int* __restrict__ conjflag, int n,
                          int L) {
  const int64_t total = int64_t(n) * L;
  for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < total;
       e += int64_t(gridDim.x) * blockDim.x) {
    const int p = int(e / L), k = int(e % L);
    cpx<TI> v = X[int64_t(k) * n + perm[p]];
    Xp[e] = {TO(v.re), conjflag[k] ? TO(-v.im) : TO(v.im)};
  }
}

template <typename TI, typename TO>
__global__ void perm_out_t(const cpx<TI>* __restrict__ Yp, cpx<TO>* __restrict__ Y,
                           const int* __restrict__ perm, const int* __restrict__ conjflag, int n,
                           int L) {
  const int64_t total = int64_t(n) * L;
  for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < total;
       e += int64_t(gridDim.x) * blockDim.x) {
    const int p = int(e / L), k = int(e % L);
    cpx<TI> v = Yp[e];
    Y[int64_t(k) * n + perm[p]] = {TO(v.re), conjflag[k] ? TO(-v.im) : TO(v.im)};
  }
}

// Per-frequency product, one workgroup (4 waves) per block, all frequency
// columns of a 64-column tile at once (lane = column).  Every slice element is
// read once per tile.
//   near block: Y_I[:, k] += sum_d f_d[k] D_d X_J[:, k]; X_J and D_d staged
//               through LDS in 64 x 64 chunks, each wave owns 16 rows
//   far block:  T = Vcat^H X_J (each wave 16 stacked columns, X_J staged
//               through LDS), T[c][k] *= f_{d(c)}[k], Y_I += Ucat T
// Accumulation into Yp with atomics.
template <typename T>
__global__ void __launch_bounds__(256) perfreq_tiled(
    const int* __restrict__ blk, const int* __restrict__ order, int nmv,
    const int* __restrict__ bterm, const int64_t* __restrict__ toff,
    const int64_t* __restrict__ tfoff, const int64_t* __restrict__ cols,
    const int* __restrict__ bcol, const cpx<T>* __restrict__ pool, const int* __restrict__ colpos,
    int L, const cpx<T>* __restrict__ Xp, cpx<T>* __restrict__ Yp) {
  __shared__ cpx<T> xs[64 * 64];
  __shared__ cpx<T> ds[64 * 64];
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const cpx<T> zero = {T(0), T(0)};
  for (int ob = blockIdx.x; ob < nmv; ob += gridDim.x) {
    const int b = order[ob];
    const int rb = blk[5 * b], m = blk[5 * b + 1] - rb, cb = blk[5 * b + 2],
              n = blk[5 * b + 3] - cb;
    const bool adm = blk[5 * b + 4] & 1;
    for (int k0 = 0; k0 < L; k0 += 64) {
      const int k = k0 + lane;
      const bool kin = k < L;
      const int kp = kin ? colpos[k] : 0;
      if (!adm) {
        for (int i0 = 0; i0 < m; i0 += 64) {
          const int in = min(64, m - i0);
          cpx<T> acc[16];
#pragma unroll
          for (int q = 0; q < 16; ++q) acc[q] = zero;
          for (int j0 = 0; j0 < n; j0 += 64) {
            const int jn = min(64, n - j0);
            __syncthreads();
            for (int e = threadIdx.x; e < jn * 64; e += 256) {
              const int jj = e >> 6, kk = e & 63;
              xs[e] = (k0 + kk < L) ? Xp[int64_t(cb + j0 + jj) * L + k0 + kk] : zero;
            }
            for (int d = bterm[b]; d < bterm[b + 1]; ++d) {
              const cpx<T>* D = pool + toff[d];
              __syncthreads();
              for (int e = threadIdx.x; e < jn * 64; e += 256) {
                const int jj = e >> 6, ii = e & 63;
                ds[e] = ii < in ? D[int64_t(j0 + jj) * m + i0 + ii] : zero;
              }
              __syncthreads();
              const cpx<T> f = kin ? pool[tfoff[d] + kp] : zero;
              cpx<T> sacc[16];
#pragma unroll
              for (int q = 0; q < 16; ++q) sacc[q] = zero;
              for (int jj = 0; jj < jn; ++jj) {
                const cpx<T> x = xs[jj * 64 + lane];
#pragma unroll
                for (int q = 0; q < 16; ++q) {
                  const cpx<T> dv = ds[jj * 64 + w * 16 + q];
                  sacc[q].re += dv.re * x.re - dv.im * x.im;
                  sacc[q].im += dv.re * x.im + dv.im * x.re;
                }
              }
#pragma unroll
              for (int q = 0; q < 16; ++q) {
                acc[q].re += f.re * sacc[q].re - f.im * sacc[q].im;
                acc[q].im += f.re * sacc[q].im + f.im * sacc[q].re;
              }
            }
          }
          if (kin) {
#pragma unroll
            for (int q = 0; q < 16; ++q) {
              const int i = w * 16 + q;
              if (i < in) {
                cpx<T>* y = Yp + int64_t(rb + i0 + i) * L + k;
                atomicAdd(&y->re, acc[q].re);
                atomicAdd(&y->im, acc[q].im);
              }
            }
          }
        }
      } else {
        const int c0 = bcol[b], c1 = bcol[b + 1];
        for (int cc = c0; cc < c1; cc += 64) {
          const int cn = min(64, c1 - cc);
          cpx<T> acc[16];
#pragma unroll
          for (int q = 0; q < 16; ++q) acc[q] = zero;
          for (int j0 = 0; j0 < n; j0 += 64) {
            const int jn = min(64, n - j0);
            __syncthreads();
            // X chunk into xs, the chunk of the stacked V columns into ds
            for (int e = threadIdx.x; e < jn * 64; e += 256) {
              const int jj = e >> 6, kk = e & 63;
              xs[e] = (k0 + kk < L) ? Xp[int64_t(cb + j0 + jj) * L + k0 + kk] : zero;
            }
            for (int e = threadIdx.x; e < cn * 64; e += 256) {
              const int cl = e >> 6, jj = e & 63;
              ds[e] = jj < jn ? pool[cols[3 * (cc + cl) + 1] + j0 + jj] : zero;
            }
            __syncthreads();
            for (int jj = 0; jj < jn; ++jj) {
              const cpx<T> x = xs[jj * 64 + lane];
#pragma unroll
              for (int q = 0; q < 16; ++q) {
                const cpx<T> v = ds[(w * 16 + q) * 64 + jj];
                acc[q].re += v.re * x.re + v.im * x.im;   // conj(v) x
                acc[q].im += v.re * x.im - v.im * x.re;
              }
            }
          }
          // scale by the fibers; T into ds
          __syncthreads();
#pragma unroll
          for (int q = 0; q < 16; ++q) {
            const int cl = w * 16 + q;
            cpx<T> t = zero;
            if (cl < cn && kin) {
              const cpx<T> f = pool[cols[3 * (cc + cl) + 2] + kp];
              t = {f.re * acc[q].re - f.im * acc[q].im, f.re * acc[q].im + f.im * acc[q].re};
            }
            ds[cl * 64 + lane] = t;
          }
          // Y_I += Ucat T: 64 rows at a time, U chunk staged into xs, 16 rows per wave
          for (int ib0 = 0; ib0 < m; ib0 += 64) {
            const int rn = min(64, m - ib0);
            __syncthreads();
            for (int e = threadIdx.x; e < cn * 64; e += 256) {
              const int cl = e >> 6, r = e & 63;
              xs[e] = r < rn ? pool[cols[3 * (cc + cl)] + ib0 + r] : zero;
            }
            __syncthreads();
            cpx<T> yacc[16];
#pragma unroll
            for (int q = 0; q < 16; ++q) yacc[q] = zero;
            for (int cl = 0; cl < cn; ++cl) {
              const cpx<T> t = ds[cl * 64 + lane];
#pragma unroll
              for (int q = 0; q < 16; ++q) {
                const cpx<T> u = xs[cl * 64 + w * 16 + q];
                yacc[q].re += u.re * t.re - u.im * t.im;
                yacc[q].im += u.re * t.im + u.im * t.re;
              }
            }
            if (kin) {
#pragma unroll
              for (int q = 0; q < 16; ++q) {
                const int r = w * 16 + q;
                if (r < rn) {
                  cpx<T>* y = Yp + int64_t(rb + ib0 + r) * L + k;
                  atomicAdd(&y->re, yacc[q].re);
                  atomicAdd(&y->im, yacc[q].im);
                }
              }
            }
          }
        }
      }
    }
  }
}

// ---- complex64 product on the matrix cores ------------------------------------
// Per far block (R stacked columns, Ubar m x R, Vbar n x R, column-major, the
// block's stack contiguous) and chunk of 64 frequency columns k:
//   T = Vbar^H X_J (R x 64), T' = F o T with F[c][k] = f_c[rep(k)],
//   Y_I += Ubar T'.
// Per near block: Y_I += sum_d f_d[rep(k)] (D_d X_J)[:, k].
// Complex products as three real v_mfma_f32_32x32x2f32 (Gauss's form; A[i][k] in lane
// i + 32 k, B[k][j] in lane j + 32 k, D[8 (r / 4) + 4 (l / 32) + r % 4][l % 32]
// in element r of lane l).  One workgroup of 4 waves per block; T' of up to
// 128 stacked columns is held in LDS, larger stacks go 128 columns at a time.
typedef float mf_v16 __attribute__((ext_vector_type(16)));

__device__ __forceinline__ mf_v16 mf_zero() {
  mf_v16 z;
#pragma unroll
  for (int r = 0; r < 16; ++r) z[r] = 0.f;
  return z;
}
__device__ __forceinline__ mf_v16 mfma32(float a, float b, mf_v16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
}

// one step of a complex product A B accumulated with three real products
// (Gauss): k1 += (a_r + a_i) b_r, k2 += a_r (b_i - b_r), k3 += a_i (b_r + b_i);
// then Re = k1 - k3, Im = k1 + k2
__device__ __forceinline__ void gauss3(cpx<float> a, cpx<float> b, mf_v16& k1, mf_v16& k2, mf_v16& k3) {
  k1 = mfma32(a.re + a.im, b.re, k1);
  k2 = mfma32(a.re, b.im - b.re, k2);
  k3 = mfma32(a.im, b.re + b.im, k3);
}

constexpr int MV_CC = 128;   // stacked columns per LDS chunk of T'
constexpr int MV_KU = 8;     // MFMA steps whose operands are loaded ahead

__global__ void __launch_bounds__(256) perfreq_mfma(
    const int* __restrict__ blk, const int* __restrict__ order, int nmv,
    const int* __restrict__ bterm, const int64_t* __restrict__ toff,
    const int64_t* __restrict__ tfoff, const int64_t* __restrict__ cols,
    const int* __restrict__ bcol, const cpx<float>* __restrict__ pool,
    const int* __restrict__ colpos, int L, const cpx<float>* __restrict__ Xp,
    cpx<float>* __restrict__ Yp) {
  __shared__ cpx<float> Ts[MV_CC * 64];
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lr = lane & 31, lh = lane >> 5;   // MFMA operand row / k-half
  for (int ob = blockIdx.x; ob < nmv; ob += gridDim.x) {
    const int b = order[ob];
    const int rb = blk[5 * b], m = blk[5 * b + 1] - rb, cb = blk[5 * b + 2],
              n = blk[5 * b + 3] - cb;
    const bool adm = blk[5 * b + 4] & 1;
    const int mt = (m + 31) >> 5;
    for (int kc = 0; kc < L; kc += 64) {
      if (!adm) {
        // near block: every wave owns output tiles (row tile, k tile)
        const int d0 = bterm[b], d1 = bterm[b + 1];
        for (int tile = w; tile < mt * 2; tile += 4) {
          const int it = tile >> 1, kt = tile & 1;
          const int kcol = kc + kt * 32 + lr;
          const bool kin = kcol < L;
          const int kp = kin ? colpos[kcol] : 0;
          const int ia = it * 32 + lr;   // A row of this lane
          mf_v16 yr = mf_zero(), yi = mf_zero();
          for (int d = d0; d < d1; ++d) {
            const cpx<float>* D = pool + toff[d];
            mf_v16 k1 = mf_zero(), k2 = mf_zero(), k3 = mf_zero();
            for (int j0 = 0; j0 < n; j0 += 2 * MV_KU) {
              // operands of MV_KU steps first, then their products
              cpx<float> a[MV_KU], x[MV_KU];
#pragma unroll
              for (int u = 0; u < MV_KU; ++u) {
                const int j = j0 + 2 * u + lh;
                a[u] = (ia < m && j < n) ? D[int64_t(j) * m + ia] : cpx<float>{0.f, 0.f};
                x[u] = (kin && j < n) ? Xp[int64_t(cb + j) * L + kcol] : cpx<float>{0.f, 0.f};
              }
#pragma unroll
              for (int u = 0; u < MV_KU; ++u) gauss3(a[u], x[u], k1, k2, k3);
            }
            const cpx<float> f = kin ? pool[tfoff[d] + kp] : cpx<float>{0.f, 0.f};
#pragma unroll
            for (int r = 0; r < 16; ++r) {
              const float pr = k1[r] - k3[r], pi = k1[r] + k2[r];
              yr[r] += f.re * pr - f.im * pi;
              yi[r] += f.re * pi + f.im * pr;
            }
          }
          if (kin) {
#pragma unroll
            for (int r = 0; r < 16; ++r) {
              const int row = it * 32 + 8 * (r >> 2) + 4 * lh + (r & 3);
              if (row < m) {
                cpx<float>* y = Yp + int64_t(rb + row) * L + kcol;
                atomicAdd(&y->re, yr[r]);
                atomicAdd(&y->im, yi[r]);
              }
            }
          }
        }
        continue;
      }
      const int c0b = bcol[b], R = bcol[b + 1] - c0b;
      if (R == 0) continue;
      const cpx<float>* Ust = pool + cols[3 * c0b];
      const cpx<float>* Vst = pool + cols[3 * c0b + 1];
      for (int cc = 0; cc < R; cc += MV_CC) {
        const int cn = min(MV_CC, R - cc);
        const int ct = (cn + 31) >> 5;
        __syncthreads();   // Ts free
        // T' = F o (Vbar^H X_J) for stacked columns cc .. cc + cn
        for (int tile = w; tile < ct * 2; tile += 4) {
          const int ti = tile >> 1, kt = tile & 1;
          const int kcol = kc + kt * 32 + lr;
          const bool kin = kcol < L;
          const int ca = cc + ti * 32 + lr;   // A row (stacked column) of this lane
          const cpx<float>* Vc = Vst + int64_t(ca) * n;
          mf_v16 k1 = mf_zero(), k2 = mf_zero(), k3 = mf_zero();
          for (int j0 = 0; j0 < n; j0 += 2 * MV_KU) {
            cpx<float> v[MV_KU], x[MV_KU];
#pragma unroll
            for (int u = 0; u < MV_KU; ++u) {
              const int j = j0 + 2 * u + lh;
              const cpx<float> vv = (ca < R && j < n) ? Vc[j] : cpx<float>{0.f, 0.f};
              v[u] = {vv.re, -vv.im};   // conj(v)
              x[u] = (kin && j < n) ? Xp[int64_t(cb + j) * L + kcol] : cpx<float>{0.f, 0.f};
            }
#pragma unroll
            for (int u = 0; u < MV_KU; ++u) gauss3(v[u], x[u], k1, k2, k3);
          }
          mf_v16 tr, tim;
#pragma unroll
          for (int r = 0; r < 16; ++r) {
            tr[r] = k1[r] - k3[r];
            tim[r] = k1[r] + k2[r];
          }
          const int kp = kin ? colpos[kcol] : 0;
#pragma unroll
          for (int r = 0; r < 16; ++r) {
            const int cl = ti * 32 + 8 * (r >> 2) + 4 * lh + (r & 3);   // local stacked column
            cpx<float> t = {0.f, 0.f};
            if (cl < cn && kin) {
              const cpx<float> f = pool[cols[3 * (c0b + cc + cl) + 2] + kp];
              t = {f.re * tr[r] - f.im * tim[r], f.re * tim[r] + f.im * tr[r]};
            }
            Ts[cl * 64 + kt * 32 + lr] = t;
          }
        }
        __syncthreads();
        // Y_I += Ubar[:, cc .. cc + cn] T'
        for (int tile = w; tile < mt * 2; tile += 4) {
          const int it = tile >> 1, kt = tile & 1;
          const int kcol = kc + kt * 32 + lr;
          const int ia = it * 32 + lr;
          mf_v16 k1 = mf_zero(), k2 = mf_zero(), k3 = mf_zero();
          for (int c2 = 0; c2 < ct * 32; c2 += 2 * MV_KU) {
            cpx<float> uu[MV_KU], tt[MV_KU];
#pragma unroll
            for (int q = 0; q < MV_KU; ++q) {
              const int cl = c2 + 2 * q + lh;   // < ct * 32 (ct * 32 is a multiple of 2 MV_KU)
              uu[q] = (ia < m && cl < cn) ? Ust[int64_t(cc + cl) * m + ia] : cpx<float>{0.f, 0.f};
              tt[q] = Ts[cl * 64 + kt * 32 + lr];
            }
#pragma unroll
            for (int q = 0; q < MV_KU; ++q) gauss3(uu[q], tt[q], k1, k2, k3);
          }
          mf_v16 yr, yi;
#pragma unroll
          for (int r = 0; r < 16; ++r) {
            yr[r] = k1[r] - k3[r];
            yi[r] = k1[r] + k2[r];
          }
          if (kcol < L) {
#pragma unroll
            for (int r = 0; r < 16; ++r) {
              const int row = it * 32 + 8 * (r >> 2) + 4 * lh + (r & 3);
              if (row < m) {
                cpx<float>* y = Yp + int64_t(rb + row) * L + kcol;
                atomicAdd(&y->re, yr[r]);
                atomicAdd(&y->im, yi[r]);
              }
            }
          }
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
    const int* __restrict__ blk, const int* __restrict__ order, int nblocks, const int* __restrict__ bterm,
    const int* __restrict__ trank, const int64_t* __restrict__ toff,
    const int64_t* __restrict__ tvoff, const int64_t* __restrict__ tfoff,
    const cpx<T>* __restrict__ pool, const int* __restrict__ colpos,
    const int* __restrict__ conjf, int L, int n,
    const cpx<T>* __restrict__ X, cpx<T>* __restrict__ ybuf, cpx<T>* __restrict__ scratch,
    int64_t sstride) {
  __shared__ cpx<T> t1[64], t2[64];
  const int lane = threadIdx.x;
  cpx<T>* w1 = scratch + int64_t(blockIdx.x) * sstride;
  for (int ob = blockIdx.x; ob < nblocks; ob += gridDim.x) {
    const int b = order[ob];   // blocks with terms, most work first
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
        const cpx<T>* V = pool + tvoff[d];
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

// the kernels of the per-frequency product on stream st (no allocation, no
// host transfer: a capturable sequence)
template <typename T>
static void enqueue_perfreq(gcq_context* ctx, hipStream_t st, int precision, const void* X, void* Y) {
  Faces3D& F = ctx->F;
  const int n = ctx->n, L = ctx->L;
  const int64_t nl = int64_t(n) * L;
  cpx<T>* Xp = F.pxy.as<cpx<T>>();
  cpx<T>* Yp = Xp + nl;
  const int* d_colpos = F.pmeta.as<int>();
  const int* d_conj = d_colpos + L;
  const int* perm = ctx->d_perm.as<int>();
  const int g = 4096;
  if (precision == GCQ_C128)
    hipLaunchKernelGGL((perm_in_t<double, T>), dim3(g), dim3(256), 0, st, (const cpx<double>*)X, Xp,
                       perm, d_conj, n, L);
  else
    hipLaunchKernelGGL((perm_in_t<float, T>), dim3(g), dim3(256), 0, st, (const cpx<float>*)X, Xp,
                       perm, d_conj, n, L);
  hipLaunchKernelGGL(zero3<T>, dim3(g), dim3(256), 0, st, Yp, nl);
  const int cus = ctx->cus;
  if constexpr (std::is_same<T, float>::value) {
    hipLaunchKernelGGL(perfreq_mfma, dim3(std::max(1, std::min(F.n_mvblocks, cus * 4))), dim3(256), 0,
                       st, ctx->d_blk.as<int>(), F.d_mvorder.as<int>(), F.n_mvblocks,
                       F.d_bterm.as<int>(), F.d_toff.as<int64_t>(), F.d_tfoff.as<int64_t>(),
                       F.d_cols.as<int64_t>(), F.d_bcol.as<int>(), F.slices.as<cpx<float>>(), d_colpos,
                       L, Xp, Yp);
  } else {
    hipLaunchKernelGGL(perfreq_tiled<T>, dim3(std::max(1, std::min(F.n_mvblocks, cus * 2))), dim3(256),
                       0, st, ctx->d_blk.as<int>(), F.d_mvorder.as<int>(), F.n_mvblocks,
                       F.d_bterm.as<int>(), F.d_toff.as<int64_t>(), F.d_tfoff.as<int64_t>(),
                       F.d_cols.as<int64_t>(), F.d_bcol.as<int>(), F.slices.as<cpx<T>>(), d_colpos, L,
                       Xp, Yp);
  }
  if (precision == GCQ_C128)
    hipLaunchKernelGGL((perm_out_t<T, double>), dim3(g), dim3(256), 0, st, Yp, (cpx<double>*)Y, perm,
                       d_conj, n, L);
  else
    hipLaunchKernelGGL((perm_out_t<T, float>), dim3(g), dim3(256), 0, st, Yp, (cpx<float>*)Y, perm,
                       d_conj, n, L);
}

// the product's buffers and frequency tables (once per operator)
static int product_setup(gcq_context* ctx, size_t need) {
  Faces3D& F = ctx->F;
  const int L = ctx->L;
  if (F.pxy.bytes < need || !F.meta_valid) {
    F.graphs.clear();   // captured graphs refer to the old buffers and tables
    GCQ_TRY(F.pxy.ensure(need));
    std::vector<int> meta(2 * L);
    for (int k = 0; k < L; ++k) {
      meta[k] = ctx->kpos[k];
      meta[L + k] = ctx->conj[k];
    }
    GCQ_TRY(upload(F.pmeta, meta, ctx->stream));
    GCQ_HIP(hipStreamSynchronize(ctx->stream));
    F.meta_valid = true;
  }
  return GCQ_OK;
}

template <typename T>
static int compressed_impl(gcq_context* ctx, int mode, int precision, const void* X, void* Y) {
  Faces3D& F = ctx->F;
  hipStream_t st = ctx->stream;
  const int n = ctx->n, L = ctx->L, nb = int(ctx->blocks.size());
  if (mode == GCQ_PER_FREQUENCY) {
    const bool bf = precision == GCQ_C64_SPLIT_BF16;
    if (bf) GCQ_TRY(bf16_setup(ctx));
    GCQ_TRY(product_setup(ctx, bf ? bf16_buffer_bytes(ctx) : size_t(2) * n * L * sizeof(cpx<T>)));
    auto enqueue = [&](hipStream_t s) {
      if (bf)
        enqueue_perfreq_bf16(ctx, s, X, Y);
      else
        enqueue_perfreq<T>(ctx, s, precision, X, Y);
    };
    if (ctx->tune.product_graph) {
      hipGraphExec_t exec = nullptr;
      for (auto& x : F.graphs.e)
        if (x.X == X && x.Y == Y && x.precision == precision) exec = x.exec;
      if (!exec) {
        if (!F.graphs.cap) GCQ_HIP(hipStreamCreateWithFlags(&F.graphs.cap, hipStreamNonBlocking));
        hipGraph_t graph = nullptr;
        GCQ_HIP(hipStreamBeginCapture(F.graphs.cap, hipStreamCaptureModeThreadLocal));
        enqueue(F.graphs.cap);
        const hipError_t ce = hipGetLastError();
        GCQ_HIP(hipStreamEndCapture(F.graphs.cap, &graph));
        if (ce != hipSuccess) {
          (void)hipGraphDestroy(graph);
          return fail(GCQ_ERR_HIP, "capture of the product failed: %s", hipGetErrorString(ce));
        }
        const hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (ie != hipSuccess) return fail(GCQ_ERR_HIP, "graph instantiation failed: %s", hipGetErrorString(ie));
        if (F.graphs.e.size() >= 8) {   // keep the most recent few
          (void)hipGraphExecDestroy(F.graphs.e.front().exec);
          F.graphs.e.erase(F.graphs.e.begin());
        }
        F.graphs.e.push_back({X, Y, precision, exec});
      }
      GCQ_TRY(timed_begin(ctx));
      GCQ_HIP(hipGraphLaunch(exec, st));
    } else {
      GCQ_TRY(timed_begin(ctx));
      enqueue(st);
    }
    GCQ_HIP(hipGetLastError());
    timed_end(ctx, "matvec_perfreq");
    return GCQ_OK;
  }
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
  const int nmv = F.n_mvblocks;
  const int wgrid = std::max(1, std::min(nmv, ctx->cus * 32));
  GCQ_TRY(ctx->scratchB.ensure(size_t(nl + n + 2 * int64_t(maxn) * wgrid) * sizeof(cpx<T>)));
  cpx<T>* Xp = ctx->scratchB.as<cpx<T>>();
  cpx<T>* Yp = Xp + nl;
  const int g = 4096;
  const int* perm = ctx->d_perm.as<int>();
  GCQ_TRY(timed_begin(ctx));
  {
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
    hipLaunchKernelGGL(wsum_kernel<T>, dim3(wgrid), dim3(64), 0, st, ctx->d_blk.as<int>(),
                       F.d_mvorder.as<int>(), nmv,
                       F.d_bterm.as<int>(), F.d_trank.as<int>(), F.d_toff.as<int64_t>(),
                       F.d_tvoff.as<int64_t>(), F.d_tfoff.as<int64_t>(), F.slices.as<cpx<T>>(),
                       d_colpos, d_conj, L, n, Xp,
                       Yp, Yp + n, int64_t(2) * maxn);
    if (precision == GCQ_C128)
      hipLaunchKernelGGL((perm_out3<T, double>), dim3(64), dim3(256), 0, st, Yp, (cpx<double>*)Y,
                         perm, ctx->scratchD.as<int>(), n, 1);
    else
      hipLaunchKernelGGL((perm_out3<T, float>), dim3(64), dim3(256), 0, st, Yp, (cpx<float>*)Y,
                         perm, ctx->scratchD.as<int>(), n, 1);
  }
  GCQ_HIP(hipGetLastError());
  timed_end(ctx, "matvec_wsum");
  return GCQ_OK;
}

// the per-frequency product's buffers and tables, ahead of a capture
int prepare_perfreq(gcq_context* ctx, int precision) {
  if (ctx->F.precision != storage_precision(precision))
    return fail(GCQ_ERR_ARG, "precision differs from the one the 3D-ACA was built in");
  const int n = ctx->n, L = ctx->L;
  if (precision == GCQ_C64_SPLIT_BF16) {
    GCQ_TRY(bf16_setup(ctx));
    return product_setup(ctx, bf16_buffer_bytes(ctx));
  }
  return product_setup(ctx, size_t(2) * n * L * (precision == GCQ_C128 ? 16 : 8));
}

// the per-frequency product's kernels on stream s (no allocation, no host
// transfer: capturable after prepare_perfreq)
void enqueue_perfreq_any(gcq_context* ctx, hipStream_t s, int precision, const void* X, void* Y,
                         const int* tile_mask) {
  if (precision == GCQ_C64_SPLIT_BF16)
    enqueue_perfreq_bf16(ctx, s, X, Y, tile_mask);
  else if (precision == GCQ_C128)
    enqueue_perfreq<double>(ctx, s, precision, X, Y);
  else
    enqueue_perfreq<float>(ctx, s, precision, X, Y);
}

int run_compressed(gcq_context* ctx, int mode, int precision, const void* X, void* Y) {
  if (ctx->F.precision != storage_precision(precision))
    return fail(GCQ_ERR_ARG, "precision differs from the one the 3D-ACA was built in");
  if (precision == GCQ_C64_SPLIT_BF16 && mode != GCQ_PER_FREQUENCY)
    return fail(GCQ_ERR_UNSUPPORTED, "split-bf16 products are per frequency only");
  return precision == GCQ_C128 ? compressed_impl<double>(ctx, mode, precision, X, Y)
                               : compressed_impl<float>(ctx, mode, precision, X, Y);
}

}  // namespace gcq
