// 3D-ACA of every block of the partition across the frequencies (Sec. 4,
// Alg. 1 with the recursive Frobenius norm of eq. norm), one wave per block.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <type_traits>

#include "internal.h"
#include "lowrank.h"
#include "near.h"

namespace gcq {

constexpr int R3_MAX = 64;      // terms per block the kernel can hold
constexpr int NK_MAX = 2048;    // frequencies in K

struct BlockDesc3 {
  int rb, m, cb, n;
  int admissible, all_far;
};

struct Term3 {
  int64_t slice;   // pool offset (elements) of the slice: dense m x n, or Ubar then Vbar
  int64_t fiber;   // pool offset of the fiber (nK elements)
  int rank;        // slice rank (far) or -1 (dense)
  int freq;        // position in K of the frequency the slice was taken at
};

template <typename T>
struct Shared3 {
  AcaShared<T> aca;
  RecompShared rs;
  cpx<double> mats[4 * 16 * 16];
  Term3 term[R3_MAX];
  cpx<T> fk[R3_MAX];          // f_d[k_cur]
  cpx<T> hp[R3_MAX];          // H_d[i_l, j_l]
  cpx<double> hin[R3_MAX];    // <H_d, H_l>
  unsigned usedk[NK_MAX / 32];
  int64_t alloc;
  int flag;
};

// pool allocation by one lane; returns -1 when the pool is exhausted
__device__ inline int64_t pool_alloc(unsigned long long* cursor, int64_t cnt, int64_t capacity) {
  unsigned long long o = atomicAdd(cursor, (unsigned long long)cnt);
  if (int64_t(o) + cnt > capacity) return -1;
  return int64_t(o);
}

// residual entry function of a far block at one frequency:
//   R(i, j) = A_ij(s) - sum_d f_d[k] (Ubar_d Vbar_d^H)[i, j]
template <typename T, bool ALLFAR>
struct ResidualEntry {
  const Tab* tab;
  int rb, cb, m, n;
  double sr, si;
  bool all_far;
  int nterm;
  Shared3<T>* sh;
  const cpx<T>* pool;
  cpx<T>* coef;   // per-wave scratch: sum_d rank_d coefficients
  bool rowmode;
  __device__ void prep_row(int i) {
    // coef[d][c] = f_d[k] Ubar_d[i][c]
    const int lane = threadIdx.x & (WAVE - 1);
    int base = 0;
    for (int d = 0; d < nterm; ++d) {
      const Term3 t = sh->term[d];
      const cpx<T>* Ud = pool + t.slice;
      for (int c = lane; c < t.rank; c += WAVE) coef[base + c] = cmul(sh->fk[d], Ud[int64_t(c) * m + i]);
      base += t.rank;
    }
    rowmode = true;
    __syncthreads();
  }
  __device__ void prep_col(int j) {
    // coef[d][c] = f_d[k] conj(Vbar_d[j][c])
    const int lane = threadIdx.x & (WAVE - 1);
    int base = 0;
    for (int d = 0; d < nterm; ++d) {
      const Term3 t = sh->term[d];
      const cpx<T>* Vd = pool + t.slice + int64_t(t.rank) * m;
      for (int c = lane; c < t.rank; c += WAVE) {
        cpx<T> v = Vd[int64_t(c) * n + j];
        coef[base + c] = cmul(sh->fk[d], cpx<T>{v.re, -v.im});
      }
      base += t.rank;
    }
    rowmode = false;
    __syncthreads();
  }
  __device__ cpx<T> operator()(int i, int j) const {
    cpx<T> a = entry<T, ALLFAR>(*tab, rb + i, cb + j, sr, si, all_far);
    int base = 0;
    for (int d = 0; d < nterm; ++d) {
      const Term3 t = sh->term[d];
      const cpx<T>* Ud = pool + t.slice;
      const cpx<T>* Vd = Ud + int64_t(t.rank) * m;
      for (int c = 0; c < t.rank; ++c) {
        cpx<T> p;
        if (rowmode) {
          cpx<T> v = Vd[int64_t(c) * n + j];
          p = cmul(coef[base + c], cpx<T>{v.re, -v.im});
        } else {
          p = cmul(Ud[int64_t(c) * m + i], coef[base + c]);
        }
        a.re -= p.re;
        a.im -= p.im;
      }
      base += t.rank;
    }
    return a;
  }
};

// entry of slice d at (i, j): dense or sum_c Ubar[i][c] conj(Vbar[j][c]) (one lane)
template <typename T>
__device__ inline cpx<T> slice_at(const Term3& t, const cpx<T>* pool, int m, int n, int i, int j) {
  if (t.rank < 0) return pool[t.slice + int64_t(j) * m + i];
  const cpx<T>* U = pool + t.slice;
  const cpx<T>* V = U + int64_t(t.rank) * m;
  cpx<T> acc = {T(0), T(0)};
  for (int c = 0; c < t.rank; ++c) {
    cpx<T> v = V[int64_t(c) * n + j];
    cpx<T> p = cmul(U[int64_t(c) * m + i], cpx<T>{v.re, -v.im});
    acc.re += p.re;
    acc.im += p.im;
  }
  return acc;
}


// Pivot of a factored slice H = Ubar Vbar^H (m x n, rank t): largest |H[i, j]|,
// first in row-major order on ties.  Each lane expands 4 x 4 tiles of the
// product (the dense block is never stored).
template <typename T>
__device__ inline void lowrank_argmax(const cpx<T>* __restrict__ U, const cpx<T>* __restrict__ V,
                                      int m, int n, int t, double& best, int& be) {
  const int lane = threadIdx.x & (WAVE - 1);
  const int ti = (m + 3) >> 2, tj = (n + 3) >> 2;
  best = -1.0;
  be = 0x7fffffff;
  for (int tile = lane; tile < ti * tj; tile += WAVE) {
    const int i0 = (tile / tj) * 4, j0 = (tile % tj) * 4;
    cpx<T> acc[4][4];
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
      for (int y = 0; y < 4; ++y) acc[x][y] = {T(0), T(0)};
    for (int c = 0; c < t; ++c) {
      cpx<T> u[4], v[4];
#pragma unroll
      for (int x = 0; x < 4; ++x) {
        u[x] = i0 + x < m ? U[int64_t(c) * m + i0 + x] : cpx<T>{T(0), T(0)};
        v[x] = j0 + x < n ? V[int64_t(c) * n + j0 + x] : cpx<T>{T(0), T(0)};
      }
#pragma unroll
      for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y) {   // u conj(v)
          acc[x][y].re += u[x].re * v[y].re + u[x].im * v[y].im;
          acc[x][y].im += u[x].im * v[y].re - u[x].re * v[y].im;
        }
    }
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
      for (int y = 0; y < 4; ++y) {
        if (i0 + x < m && j0 + y < n) {
          const double val = mag2(acc[x][y]);
          const int e = (i0 + x) * n + j0 + y;
          if (val > best || (val == best && e < be)) { best = val; be = e; }
        }
      }
  }
  wave_argmax(best, be);
}

// <H_d, H_l>_F = sum_{a,b} (U_l^H U_d)[a][b] (V_d^H V_l)[b][a] for factored
// slices; lanes own (a, b) pairs, rows are staged through LDS R at a time.
// stage: LDS scratch of 16 KB (2 * 64 * R elements).
template <typename T>
__device__ inline cpx<double> lowrank_inner(const cpx<T>* __restrict__ Ul, const cpx<T>* __restrict__ Vl,
                                            int tl, const cpx<T>* __restrict__ Ud,
                                            const cpx<T>* __restrict__ Vd, int td, int m, int n,
                                            cpx<T>* stage) {
  constexpr int R = int(128 / sizeof(cpx<T>));   // 16 (float) or 8 (double)
  const int lane = threadIdx.x & (WAVE - 1);
  cpx<T>* sl = stage;           // [a][r]
  cpx<T>* sd = stage + 64 * R;  // [b][r]
  double re = 0.0, im = 0.0;
  for (int p0 = 0; p0 < tl * td; p0 += WAVE) {
    const int p = p0 + lane;
    const bool act = p < tl * td;
    const int a = act ? p / td : 0, b = act ? p % td : 0;
    double pr = 0, pi = 0, qr = 0, qi = 0;
    for (int side = 0; side < 2; ++side) {
      const int len = side == 0 ? m : n;
      const cpx<T>* X = side == 0 ? Ul : Vd;   // conjugated operand
      const cpx<T>* Y = side == 0 ? Ud : Vl;
      const int tx = side == 0 ? tl : td, ty = side == 0 ? td : tl;
      const int ax = side == 0 ? a : b, ay = side == 0 ? b : a;
      double sr = 0, si = 0;
      for (int r0 = 0; r0 < len; r0 += R) {
        const int rn = min(R, len - r0);
        __syncthreads();
        for (int e = lane; e < tx * R; e += WAVE) {
          const int c = e / R, r = e % R;
          sl[e] = r < rn ? X[int64_t(c) * len + r0 + r] : cpx<T>{T(0), T(0)};
        }
        for (int e = lane; e < ty * R; e += WAVE) {
          const int c = e / R, r = e % R;
          sd[e] = r < rn ? Y[int64_t(c) * len + r0 + r] : cpx<T>{T(0), T(0)};
        }
        __syncthreads();
        if (act) {
#pragma unroll 4
          for (int r = 0; r < R; ++r) {
            const cpx<T> x = sl[ax * R + r], y = sd[ay * R + r];
            sr += double(x.re) * y.re + double(x.im) * y.im;   // conj(x) y
            si += double(x.re) * y.im - double(x.im) * y.re;
          }
        }
      }
      if (side == 0) { pr = sr; pi = si; } else { qr = sr; qi = si; }
    }
    if (act) {
      re += pr * qr - pi * qi;
      im += pr * qi + pi * qr;
    }
  }
  __syncthreads();
  return {wave_sum(re), wave_sum(im)};
}

// ALLFAR = true: admissible blocks without self/near-tier entries (the float64
// quadrature tiers are not compiled in); ALLFAR = false: every other block.
template <typename T, bool ALLFAR>
__global__ void __launch_bounds__(64) aca3d_kernel(
    Tab tab, const BlockDesc3* __restrict__ blocks, const int* __restrict__ order, int nblocks,
    const double2* __restrict__ sigK, int nK, double tol_aca, double tol, int rmax, int aca_cap,
    unsigned char* __restrict__ ws, int64_t ws_stride, cpx<T>* __restrict__ pool,
    unsigned long long* __restrict__ cursor, int64_t capacity, Term3* __restrict__ terms,
    int* __restrict__ brank, int* __restrict__ bstatus, int* __restrict__ counter) {
  __shared__ Shared3<T> sh;
  const int lane = threadIdx.x;
  unsigned char* myws = ws + int64_t(blockIdx.x) * ws_stride;
  // per-wave scratch layout: ACA workspace, Jacobi matrices, residual coefficients
  for (;;) {
    int idx = 0;
    if (lane == 0) idx = atomicAdd(counter, 1);
    idx = __shfl(idx, 0, WAVE);
    if (idx >= nblocks) break;
    const int b = order[idx];
    const BlockDesc3 B = blocks[b];
    const int m = B.m, n = B.n;
    const int cap = min(min(m, n), aca_cap);
    cpx<T>* U = reinterpret_cast<cpx<T>*>(myws);
    cpx<T>* W = U + int64_t(cap) * m;
    cpx<double>* GU = reinterpret_cast<cpx<double>*>(myws + ws_gram_off<T>(cap, m, n));
    cpx<double>* GV = GU + cap * cap;
    cpx<double>* jmats = reinterpret_cast<cpx<double>*>(myws + ws_bytes<T>(cap, m, n));
    cpx<T>* coef = reinterpret_cast<cpx<T>*>(jmats + 4 * 64 * 64);
    // Gram matrix <H_d, H_d'> of the accepted slices (R3_MAX x R3_MAX)
    cpx<double>* G3 = reinterpret_cast<cpx<double>*>(coef + R3_MAX * 64);
    for (int w = lane; w < (nK + 31) / 32; w += WAVE) sh.usedk[w] = 0u;
    __syncthreads();
    int ell = 0, kcur = 0, status = 0;
    double norm2 = 0.0;
    while (true) {
      for (int d = lane; d < ell; d += WAVE) sh.fk[d] = pool[sh.term[d].fiber + kcur];
      __syncthreads();
      const double2 sg = sigK[kcur];
      int64_t soff = -1;
      int srank = -1;
      // ---- residual slice at k_cur
      if (!ALLFAR && !B.admissible) {
        if (lane == 0) sh.alloc = pool_alloc(cursor, int64_t(m) * n, capacity);
        __syncthreads();
        soff = sh.alloc;
        if (soff < 0) { status |= ST_DEFERRED; break; }
        for (int e = lane; e < m * n; e += WAVE) {
          const int r = e % m, c = e / m;
          cpx<T> a = entry<T, ALLFAR>(tab, B.rb + r, B.cb + c, sg.x, sg.y, B.all_far != 0);
          for (int d = 0; d < ell; ++d) {
            cpx<T> p = cmul(sh.fk[d], pool[sh.term[d].slice + e]);
            a.re -= p.re;
            a.im -= p.im;
          }
          pool[soff + e] = a;
        }
      } else {
        ResidualEntry<T, ALLFAR> ent{&tab, B.rb, B.cb, m, n, sg.x, sg.y, B.all_far != 0, ell, &sh,
                                     pool, coef, true};
        // nu = |sum_d f_d[k] H_d|_F, the current approximation of the block at
        // k: the slice tolerance is taken relative to max(|residual|, nu)
        double nu2 = 0.0;
        for (int e = lane; e < ell * ell; e += WAVE) {
          const int d = e / ell, d2 = e % ell;
          const cpx<T> a = sh.fk[d], b = sh.fk[d2];
          const cpx<double> g = G3[d * R3_MAX + d2];
          // a conj(b) <H_d, H_d2>
          const double pr = double(a.re) * b.re + double(a.im) * b.im;
          const double pi = double(a.im) * b.re - double(a.re) * b.im;
          nu2 += pr * g.re - pi * g.im;
        }
        const double nu = sqrt(fmax(wave_sum(nu2), 0.0));
        int ast = 0;
        const int k = aca_wave<T>(ent, m, n, cap, aca_cap, tol_aca, nu, U, W, GU, GV, sh.aca, ast);
        if (ast & ST_CAPPED) status |= ST_CAPPED;
        cpx<double>* A = k <= 16 ? sh.mats : jmats;
        const int t = recompress_wave(k, cap, GU, GV, tol_aca, nu, true, A, sh.rs);
        if (lane == 0) sh.alloc = pool_alloc(cursor, int64_t(t) * (m + n), capacity);
        __syncthreads();
        soff = sh.alloc;
        if (soff < 0) { status |= ST_DEFERRED; break; }
        apply_factors<T>(k, t, m, n, U, W, GU, GV, pool + soff, pool + soff + int64_t(t) * m, lane,
                         WAVE);
        srank = t;
      }
      __syncthreads();
      Term3 cur;
      cur.slice = soff;
      cur.rank = srank;
      cur.freq = kcur;
      // ---- pivot: largest modulus, first in row-major order on ties
      double best = -1.0;
      int be = 0x7fffffff;
      const int mn = m * n;
      if (srank >= 0) {
        lowrank_argmax<T>(pool + soff, pool + soff + int64_t(srank) * m, m, n, srank, best, be);
      } else {
        for (int e = lane; e < mn; e += WAVE) {
          const int i = e / n, j = e % n;  // row-major key
          cpx<T> h = slice_at<T>(cur, pool, m, n, i, j);
          double v = mag2(h);
          if (v > best) { best = v; be = e; }
        }
        wave_argmax(best, be);
      }
      if (!(best > PivFloor<T>::v)) break;   // zero pivot: rank stays ell
      const int ip = be / n, jp = be % n;
      const cpx<T> piv = slice_at<T>(cur, pool, m, n, ip, jp);
      for (int d = lane; d < ell; d += WAVE) sh.hp[d] = slice_at<T>(sh.term[d], pool, m, n, ip, jp);
      if (lane == 0) sh.alloc = pool_alloc(cursor, nK, capacity);
      __syncthreads();
      const int64_t foff = sh.alloc;
      if (foff < 0) { status |= ST_DEFERRED; break; }
      cur.fiber = foff;
      // ---- fiber over K
      const cpx<T> inv = cinv(piv);
      double nf2 = 0.0;
      for (int kk = lane; kk < nK; kk += WAVE) {
        const double2 s2 = sigK[kk];
        cpx<T> a = entry<T, ALLFAR>(tab, B.rb + ip, B.cb + jp, s2.x, s2.y, B.all_far != 0);
        for (int d = 0; d < ell; ++d) {
          cpx<T> p = cmul(sh.hp[d], pool[sh.term[d].fiber + kk]);
          a.re -= p.re;
          a.im -= p.im;
        }
        cpx<T> f = (kk == kcur && B.admissible == 0) ? cpx<T>{T(1), T(0)} : cmul(a, inv);
        pool[foff + kk] = f;
        nf2 += double(f.re) * double(f.re) + double(f.im) * double(f.im);
      }
      __syncthreads();
      nf2 = wave_sum(nf2);
      // ---- eq. norm: <H_d, H_l> <f_d, f_l> cross terms and |H_l|^2 |f_l|^2
      double nh2 = 0.0;
      if (!ALLFAR && !B.admissible) {
        for (int e = lane; e < mn; e += WAVE) {
          cpx<T> h = pool[soff + e];
          nh2 += double(h.re) * double(h.re) + double(h.im) * double(h.im);
        }
        nh2 = wave_sum(nh2);
        for (int d = 0; d < ell; ++d) {
          double re = 0, im = 0;
          const cpx<T>* Hd = pool + sh.term[d].slice;
          for (int e = lane; e < mn; e += WAVE) {
            cpx<T> x = Hd[e], y = pool[soff + e];
            re += double(x.re) * y.re + double(x.im) * y.im;   // x conj(y)
            im += double(x.im) * y.re - double(x.re) * y.im;
          }
          re = wave_sum(re);
          im = wave_sum(im);
          if (lane == 0) sh.hin[d] = {re, im};
        }
      } else {
        // <H_d, H_l> = tr((U_l^H U_d)(V_d^H V_l)); |H_l|^2 likewise with d = l
        const int tl = srank;
        const cpx<T>* Ul = pool + soff;
        const cpx<T>* Vl = Ul + int64_t(tl) * m;
        cpx<T>* stage = reinterpret_cast<cpx<T>*>(sh.mats);
        for (int d = 0; d <= ell; ++d) {
          const Term3 td = d < ell ? sh.term[d] : cur;
          const cpx<T>* Ud = pool + td.slice;
          const cpx<T>* Vd = Ud + int64_t(td.rank) * m;
          const cpx<double> h = lowrank_inner<T>(Ul, Vl, tl, Ud, Vd, td.rank, m, n, stage);
          if (d < ell) {
            if (lane == 0) sh.hin[d] = h;
          } else {
            nh2 = h.re;
          }
        }
      }
      __syncthreads();
      double cross = 0.0;
      for (int d = 0; d < ell; ++d) {
        double fr = 0, fi = 0;  // <f_d, f_l> = sum f_d conj(f_l)
        for (int kk = lane; kk < nK; kk += WAVE) {
          cpx<T> x = pool[sh.term[d].fiber + kk], y = pool[foff + kk];
          fr += double(x.re) * y.re + double(x.im) * y.im;
          fi += double(x.im) * y.re - double(x.re) * y.im;
        }
        fr = wave_sum(fr);
        fi = wave_sum(fi);
        cross += sh.hin[d].re * fr - sh.hin[d].im * fi;
      }
      norm2 += 2.0 * cross + nh2 * nf2;
      if (lane == 0) sh.usedk[kcur >> 5] |= 1u << (kcur & 31);
      __syncthreads();
      if (sqrt(fmax(nh2 * nf2, 0.0)) <= tol * sqrt(fmax(norm2, 0.0))) break;  // drop term l
      if (lane == 0) sh.term[ell] = cur;
      for (int d = lane; d <= ell; d += WAVE) {
        // <H_d, H_l> (d < l) and |H_l|^2
        const cpx<double> h = d < ell ? sh.hin[d] : cpx<double>{nh2, 0.0};
        G3[d * R3_MAX + ell] = h;
        G3[ell * R3_MAX + d] = {h.re, -h.im};
      }
      __syncthreads();
      ++ell;
      // next frequency: largest |f_l[k]| among unused k (lowest k on ties)
      double bf = -1.0;
      int bk = 0x7fffffff;
      for (int kk = lane; kk < nK; kk += WAVE) {
        if ((sh.usedk[kk >> 5] >> (kk & 31)) & 1u) continue;
        double v = mag2(pool[foff + kk]);
        if (v > bf) { bf = v; bk = kk; }
      }
      wave_argmax(bf, bk);
      if (bk == 0x7fffffff) break;                       // every frequency used
      if (ell >= rmax) { status |= ST_CAPPED; break; }
      if (!(bf > 0.0)) break;                            // fiber zero at all unused ones
      kcur = bk;
    }
    __syncthreads();
    for (int d = lane; d < ell; d += WAVE) terms[int64_t(b) * R3_MAX + d] = sh.term[d];
    if (lane == 0) {
      brank[b] = ell;
      bstatus[b] = status;
    }
    __syncthreads();
  }
}


// 3D-ACA of an inadmissible block from its precomputed entry tensor
// Cn[k * stride + base + e] (all frequencies of K): the residual slices, the
// pivots and the fibers are read instead of re-evaluated.  One wave per block.
template <typename T>
struct SharedN {
  Term3 term[R3_MAX];
  cpx<T> fk[R3_MAX];
  cpx<T> hp[R3_MAX];
  cpx<double> hin[R3_MAX];
  unsigned usedk[NK_MAX / 32];
  int64_t alloc;
};

template <typename T>
__global__ void __launch_bounds__(64) aca3d_near_kernel(
    const BlockDesc3* __restrict__ blocks, const int* __restrict__ qlist, int nq,
    const int* __restrict__ near_ids, const int64_t* __restrict__ near_off, int64_t base0,
    const cpx<T>* __restrict__ Cn, int64_t stride, int nK, double tol, int rmax,
    cpx<T>* __restrict__ pool, unsigned long long* __restrict__ cursor, int64_t capacity,
    Term3* __restrict__ terms, int* __restrict__ brank, int* __restrict__ bstatus,
    int* __restrict__ counter) {
  __shared__ SharedN<T> sh;
  const int lane = threadIdx.x;
  for (;;) {
    int idx = 0;
    if (lane == 0) idx = atomicAdd(counter, 1);
    idx = __shfl(idx, 0, WAVE);
    if (idx >= nq) break;
    const int q = qlist[idx];
    const int b = near_ids[q];
    const BlockDesc3 B = blocks[b];
    const int m = B.m, n = B.n, mn = m * n;
    const int64_t base = near_off[q] - base0;
    for (int w = lane; w < (nK + 31) / 32; w += WAVE) sh.usedk[w] = 0u;
    __syncthreads();
    int ell = 0, kcur = 0, status = 0;
    double norm2 = 0.0;
    while (true) {
      for (int d = lane; d < ell; d += WAVE) sh.fk[d] = pool[sh.term[d].fiber + kcur];
      if (lane == 0) sh.alloc = pool_alloc(cursor, int64_t(mn), capacity);
      __syncthreads();
      const int64_t soff = sh.alloc;
      if (soff < 0) { status |= ST_DEFERRED; break; }
      // residual slice at k_cur and its norm
      const cpx<T>* Ck = Cn + int64_t(kcur) * stride + base;
      double nh2 = 0.0;
      for (int e = lane; e < mn; e += WAVE) {
        cpx<T> a = Ck[e];
        for (int d = 0; d < ell; ++d) {
          cpx<T> p = cmul(sh.fk[d], pool[sh.term[d].slice + e]);
          a.re -= p.re;
          a.im -= p.im;
        }
        pool[soff + e] = a;
        nh2 += mag2(a);
      }
      nh2 = wave_sum(nh2);
      __syncthreads();
      // pivot: largest modulus, first in row-major order on ties
      double best = -1.0;
      int be = 0x7fffffff;
      for (int e = lane; e < mn; e += WAVE) {
        const int i = e / n, j = e % n;
        const double v = mag2(pool[soff + int64_t(j) * m + i]);
        if (v > best) { best = v; be = e; }
      }
      wave_argmax(best, be);
      if (!(best > PivFloor<T>::v)) break;
      const int ip = be / n, jp = be % n;
      const int64_t ep = int64_t(jp) * m + ip;
      const cpx<T> piv = pool[soff + ep];
      for (int d = lane; d < ell; d += WAVE) sh.hp[d] = pool[sh.term[d].slice + ep];
      if (lane == 0) sh.alloc = pool_alloc(cursor, nK, capacity);
      __syncthreads();
      const int64_t foff = sh.alloc;
      if (foff < 0) { status |= ST_DEFERRED; break; }
      const cpx<T> inv = cinv(piv);
      double nf2 = 0.0;
      for (int kk = lane; kk < nK; kk += WAVE) {
        cpx<T> a = Cn[int64_t(kk) * stride + base + ep];
        for (int d = 0; d < ell; ++d) {
          cpx<T> p = cmul(sh.hp[d], pool[sh.term[d].fiber + kk]);
          a.re -= p.re;
          a.im -= p.im;
        }
        const cpx<T> f = kk == kcur ? cpx<T>{T(1), T(0)} : cmul(a, inv);
        pool[foff + kk] = f;
        nf2 += mag2(f);
      }
      nf2 = wave_sum(nf2);
      __syncthreads();
      // eq. norm cross terms
      double cross = 0.0;
      for (int d = 0; d < ell; ++d) {
        double hr = 0, hi = 0, fr = 0, fi = 0;
        const cpx<T>* Hd = pool + sh.term[d].slice;
        for (int e = lane; e < mn; e += WAVE) {
          const cpx<T> x = Hd[e], y = pool[soff + e];
          hr += double(x.re) * y.re + double(x.im) * y.im;   // x conj(y)
          hi += double(x.im) * y.re - double(x.re) * y.im;
        }
        const cpx<T>* fd = pool + sh.term[d].fiber;
        for (int kk = lane; kk < nK; kk += WAVE) {
          const cpx<T> x = fd[kk], y = pool[foff + kk];
          fr += double(x.re) * y.re + double(x.im) * y.im;
          fi += double(x.im) * y.re - double(x.re) * y.im;
        }
        hr = wave_sum(hr);
        hi = wave_sum(hi);
        fr = wave_sum(fr);
        fi = wave_sum(fi);
        cross += hr * fr - hi * fi;
      }
      norm2 += 2.0 * cross + nh2 * nf2;
      if (lane == 0) sh.usedk[kcur >> 5] |= 1u << (kcur & 31);
      __syncthreads();
      if (sqrt(fmax(nh2 * nf2, 0.0)) <= tol * sqrt(fmax(norm2, 0.0))) break;
      if (lane == 0) {
        Term3 t;
        t.slice = soff;
        t.fiber = foff;
        t.rank = -1;
        t.freq = kcur;
        sh.term[ell] = t;
      }
      __syncthreads();
      ++ell;
      double bf = -1.0;
      int bk = 0x7fffffff;
      for (int kk = lane; kk < nK; kk += WAVE) {
        if ((sh.usedk[kk >> 5] >> (kk & 31)) & 1u) continue;
        const double v = mag2(pool[foff + kk]);
        if (v > bf) { bf = v; bk = kk; }
      }
      wave_argmax(bf, bk);
      if (bk == 0x7fffffff) break;                       // every frequency used
      if (ell >= rmax) { status |= ST_CAPPED; break; }
      if (!(bf > 0.0)) break;                            // fiber zero at all unused ones
      kcur = bk;
    }
    __syncthreads();
    for (int d = lane; d < ell; d += WAVE) terms[int64_t(b) * R3_MAX + d] = sh.term[d];
    if (lane == 0) {
      brank[b] = ell;
      bstatus[b] = status;
    }
    __syncthreads();
  }
}

static __global__ void zero_int_3d(int* p, int n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

}  // namespace gcq

using namespace gcq;

extern "C" GCQ_API int gcq_aca3d(gcq_context* ctx, double tol_aca, double tol,
                                 int32_t max_freq_rank, int32_t precision, uint32_t flags,
                                 gcq_aca3d_stats* stats) {
  (void)flags;
  if (!ctx) return fail(GCQ_ERR_ARG, "ctx is NULL");
  GCQ_NEED_DEVICE(ctx);
  if (!ctx->have_tree || !ctx->have_freq)
    return fail(GCQ_ERR_STATE, "upload mesh, frequencies and build the tree first");
  if (precision != GCQ_C128 && precision != GCQ_C64)
    return fail(GCQ_ERR_ARG, "unknown precision %d", precision);
  if (!(tol_aca >= 0.0) || !(tol >= 0.0)) return fail(GCQ_ERR_ARG, "tolerances must be >= 0");
  if (max_freq_rank < 1 || max_freq_rank > R3_MAX)
    return fail(GCQ_ERR_ARG, "max_freq_rank must be in 1..%d", R3_MAX);
  const int nK = int(ctx->K.size());
  if (nK > NK_MAX) return fail(GCQ_ERR_UNSUPPORTED, "more than %d distinct frequencies", NK_MAX);
  GCQ_HIP(hipSetDevice(ctx->device));
  Faces3D& F = ctx->F;
  F.valid = false;
  F.precision = precision;
  F.nK = nK;
  const int nb = int(ctx->blocks.size());
  std::vector<BlockDesc3> bd(nb);
  int maxm = 0, maxmn = 0;
  for (int b = 0; b < nb; ++b) {
    const Block& B = ctx->blocks[b];
    const Cluster& A = ctx->clusters[B.row];
    const Cluster& C = ctx->clusters[B.col];
    bd[b] = {A.begin, A.end - A.begin, C.begin, C.end - C.begin, B.admissible ? 1 : 0,
             B.all_far ? 1 : 0};
    if (bd[b].m > ACA_MAXM) return fail(GCQ_ERR_UNSUPPORTED, "block too large");
    if (B.admissible) maxmn = std::max(maxmn, bd[b].m + bd[b].n);
    maxm = std::max(maxm, bd[b].m);
  }
  // work list: most expensive blocks first
  std::vector<int> order(nb);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    auto cost = [&](int x) {
      return bd[x].admissible ? double(bd[x].m) * bd[x].n * 4.0 : double(bd[x].m) * bd[x].n;
    };
    return cost(a) > cost(b);
  });
  std::vector<double2> sig(nK);
  for (int p = 0; p < nK; ++p) {
    std::complex<double> s = ctx->s[ctx->K[p]] / ctx->c;
    sig[p] = make_double2(s.real(), s.imag());
  }
  const int aca_cap = 64;
  const int64_t csz = csize(precision);
  const int64_t ws_stride =
      ((precision == GCQ_C128 ? ws_bytes<double>(aca_cap, maxmn, 0) : ws_bytes<float>(aca_cap, maxmn, 0)) +
       int64_t(4) * 64 * 64 * 16 + int64_t(R3_MAX) * 64 * csz + int64_t(R3_MAX) * R3_MAX * 16 +
       4095) & ~int64_t(4095);
  int cus = 256;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, ctx->device) == hipSuccess) cus = prop.multiProcessorCount;
  const int grid = std::min(nb, cus * 8);
  GCQ_TRY(ctx->scratchA.ensure(size_t(ws_stride) * grid));
  // pool: dense near slices and factored far slices, bump-allocated
  size_t freeb = 0, totalb = 0;
  GCQ_HIP(hipMemGetInfo(&freeb, &totalb));
  int64_t near_elems = 0, far_dims = 0;
  for (int b = 0; b < nb; ++b)
    if (bd[b].admissible) far_dims += bd[b].m + bd[b].n;
    else near_elems += int64_t(bd[b].m) * bd[b].n;
  // expected need: dense slices (near) and factored slices (far) of ~max_freq_rank/2
  // terms each, plus one fiber per term
  const int64_t rexp = std::max(8, int(max_freq_rank) / 2 + 4);
  int64_t want = near_elems * rexp + far_dims * 16 * rexp + int64_t(nb) * rexp * nK;
  int64_t capacity = std::min<int64_t>(want, int64_t(double(freeb) * 0.5) / csz);
  F.slices.release();
  GCQ_TRY(F.slices.ensure(size_t(capacity) * csz + 256));
  std::vector<int32_t> blkrank(nb), blkstat(nb);
  std::vector<Term3> terms(size_t(nb) * R3_MAX);
  GCQ_TRY(upload(ctx->scratchB, bd, ctx->stream));
  GCQ_TRY(upload(ctx->scratchC, sig, ctx->stream));
  // scratch layout: cursor (8 B), 8 counters, terms, ranks, status, work order
  GCQ_TRY(ctx->scratchD.ensure(64 + sizeof(Term3) * size_t(nb) * R3_MAX + sizeof(int) * 3 * size_t(nb)));
  unsigned long long* d_cursor = ctx->scratchD.as<unsigned long long>();
  int* d_counter = reinterpret_cast<int*>(ctx->scratchD.as<unsigned char>() + 16);
  Term3* d_terms = reinterpret_cast<Term3*>(ctx->scratchD.as<unsigned char>() + 64);
  int* d_rank = reinterpret_cast<int*>(d_terms + size_t(nb) * R3_MAX);
  int* d_stat = d_rank + nb;
  int* d_order = d_stat + nb;
  GCQ_HIP(hipMemcpyAsync(d_order, order.data(), sizeof(int) * nb, hipMemcpyHostToDevice,
                         ctx->stream));
  int64_t used = 0;
  double ms = 0.0, ms_far = 0.0, ms_near = 0.0, ms_tensor = 0.0;
  int rounds = 0;
  std::vector<int> near_pos(nb, -1);
  for (size_t q = 0; q < ctx->near_ids.size(); ++q) near_pos[ctx->near_ids[q]] = int(q);
  // element offsets of the self/near-tier entries, for batching
  std::vector<int64_t> sing_off(ctx->n_sing);
  if (ctx->n_sing > 0) {
    std::vector<SingEntry> sl(ctx->n_sing);
    GCQ_HIP(hipMemcpy(sl.data(), ctx->d_sing.p, sizeof(SingEntry) * ctx->n_sing, hipMemcpyDeviceToHost));
    for (int64_t a = 0; a < ctx->n_sing; ++a) sing_off[a] = sl[a].off;
  }
  DevBuf tensor;
  const int64_t tensor_budget = std::max<int64_t>(int64_t(1) << 28,
                                                  std::min<int64_t>(int64_t(48) << 30, int64_t(double(freeb) * 0.25)));
  std::vector<int> todo = order;
  for (int round = 0; round < 4 && !todo.empty(); ++round) {
    hipLaunchKernelGGL(zero_int_3d, dim3(1), dim3(64), 0, ctx->stream, d_counter, 8);
    unsigned long long cur0 = (unsigned long long)used;
    GCQ_HIP(hipMemcpyAsync(d_cursor, &cur0, sizeof(cur0), hipMemcpyHostToDevice, ctx->stream));
    // admissible blocks without near-tier entries, other admissible blocks,
    // inadmissible blocks (from their entry tensor)
    std::vector<int> lf, lo, lq;
    for (int b : todo) {
      if (bd[b].admissible) (bd[b].all_far ? lf : lo).push_back(b);
      else lq.push_back(near_pos[b]);
    }
    std::sort(lq.begin(), lq.end());
    std::vector<int> both(lf);
    both.insert(both.end(), lo.begin(), lo.end());
    both.insert(both.end(), lq.begin(), lq.end());
    GCQ_HIP(hipMemcpyAsync(d_order, both.data(), sizeof(int) * both.size(), hipMemcpyHostToDevice,
                           ctx->stream));
    GCQ_TRY(timed_begin(ctx));
    auto launch = [&](auto tag_t, auto tag_a, int off, int cnt, int* ctr) {
      using TT = decltype(tag_t);
      constexpr bool AA = decltype(tag_a)::value;
      if (cnt == 0) return;
      hipLaunchKernelGGL((aca3d_kernel<TT, AA>), dim3(std::min(grid, cnt)), dim3(64), 0,
                         ctx->stream, ctx->tab(), ctx->scratchB.as<BlockDesc3>(), d_order + off,
                         cnt, ctx->scratchC.as<double2>(), nK, tol_aca, tol, int(max_freq_rank),
                         aca_cap, ctx->scratchA.as<unsigned char>(), ws_stride,
                         F.slices.as<cpx<TT>>(), d_cursor, capacity, d_terms, d_rank, d_stat, ctr);
    };
    using TrueT = std::integral_constant<bool, true>;
    using FalseT = std::integral_constant<bool, false>;
    if (precision == GCQ_C128) {
      launch(double(0), TrueT(), 0, int(lf.size()), d_counter);
      launch(double(0), FalseT(), int(lf.size()), int(lo.size()), d_counter + 1);
    } else {
      launch(float(0), TrueT(), 0, int(lf.size()), d_counter);
      launch(float(0), FalseT(), int(lf.size()), int(lo.size()), d_counter + 1);
    }
    GCQ_HIP(hipGetLastError());
    ms_far += timed_end(ctx, "aca3d_far_round");
    // inadmissible blocks in batches whose entry tensor fits the budget
    size_t pos = 0;
    const int* d_q = d_order + lf.size() + lo.size();
    while (pos < lq.size()) {
      const int q0 = lq[pos];
      size_t end = pos;
      while (end < lq.size() &&
             (ctx->near_off[lq[end]] + int64_t(bd[ctx->near_ids[lq[end]]].m) * bd[ctx->near_ids[lq[end]]].n -
              ctx->near_off[q0]) * nK * csz <= tensor_budget)
        ++end;
      if (end == pos) end = pos + 1;
      const int q1 = lq[end - 1] + 1;
      const int64_t base0 = ctx->near_off[q0];
      const int64_t span = (q1 < int(ctx->near_off.size()) ? ctx->near_off[q1] : ctx->near_total) - base0;
      GCQ_TRY(tensor.ensure(size_t(span) * nK * csz + 256));
      // self/near-tier entries of [q0, q1)
      const int64_t s0 = int64_t(std::lower_bound(sing_off.begin(), sing_off.end(), base0) - sing_off.begin());
      const int64_t s1 = int64_t(std::lower_bound(sing_off.begin(), sing_off.end(), base0 + span) - sing_off.begin());
      GCQ_TRY(timed_begin(ctx));
      const dim3 g1(std::min(q1 - q0, 65536)), g2(4096);
      hipLaunchKernelGGL(zero_int_3d, dim3(1), dim3(64), 0, ctx->stream, d_counter + 2, 1);
      if (precision == GCQ_C128) {
        hipLaunchKernelGGL(near_far_tier<double>, g1, dim3(256), 0, ctx->stream, ctx->tab(),
                           ctx->d_blk.as<int>(), ctx->d_near_ids.as<int>(),
                           ctx->d_near_off.as<int64_t>(), q0, q1, base0,
                           ctx->scratchC.as<double2>(), nK, tensor.as<cpx<double>>(), span);
        hipLaunchKernelGGL(near_sing<double>, g2, dim3(256), 0, ctx->stream, ctx->tab(),
                           ctx->d_sing.as<SingEntry>(), s0, s1, base0, ctx->scratchC.as<double2>(),
                           nK, tensor.as<cpx<double>>(), span);
      } else {
        hipLaunchKernelGGL(near_far_tier<float>, g1, dim3(256), 0, ctx->stream, ctx->tab(),
                           ctx->d_blk.as<int>(), ctx->d_near_ids.as<int>(),
                           ctx->d_near_off.as<int64_t>(), q0, q1, base0,
                           ctx->scratchC.as<double2>(), nK, tensor.as<cpx<float>>(), span);
        hipLaunchKernelGGL(near_sing<float>, g2, dim3(256), 0, ctx->stream, ctx->tab(),
                           ctx->d_sing.as<SingEntry>(), s0, s1, base0, ctx->scratchC.as<double2>(),
                           nK, tensor.as<cpx<float>>(), span);
      }
      GCQ_HIP(hipGetLastError());
      ms_tensor += timed_end(ctx, "aca3d_tensor_batch");
      GCQ_TRY(timed_begin(ctx));
      const int cnt = int(end - pos);
      if (precision == GCQ_C128)
        hipLaunchKernelGGL(aca3d_near_kernel<double>, dim3(std::min(cnt, cus * 16)), dim3(64), 0,
                           ctx->stream, ctx->scratchB.as<BlockDesc3>(), d_q + pos, cnt,
                           ctx->d_near_ids.as<int>(), ctx->d_near_off.as<int64_t>(), base0,
                           tensor.as<cpx<double>>(), span, nK, tol, int(max_freq_rank),
                           F.slices.as<cpx<double>>(), d_cursor, capacity, d_terms, d_rank,
                           d_stat, d_counter + 2);
      else
        hipLaunchKernelGGL(aca3d_near_kernel<float>, dim3(std::min(cnt, cus * 16)), dim3(64), 0,
                           ctx->stream, ctx->scratchB.as<BlockDesc3>(), d_q + pos, cnt,
                           ctx->d_near_ids.as<int>(), ctx->d_near_off.as<int64_t>(), base0,
                           tensor.as<cpx<float>>(), span, nK, tol, int(max_freq_rank),
                           F.slices.as<cpx<float>>(), d_cursor, capacity, d_terms, d_rank,
                           d_stat, d_counter + 2);
      GCQ_HIP(hipGetLastError());
      ms_near += timed_end(ctx, "aca3d_near_batch");
      pos = end;
    }
    ms = ms_far + ms_tensor + ms_near;
    ++rounds;
    GCQ_HIP(hipGetLastError());
    unsigned long long curh = 0;
    GCQ_HIP(hipMemcpy(&curh, d_cursor, sizeof(curh), hipMemcpyDeviceToHost));
    GCQ_HIP(hipMemcpy(blkrank.data(), d_rank, sizeof(int) * nb, hipMemcpyDeviceToHost));
    GCQ_HIP(hipMemcpy(blkstat.data(), d_stat, sizeof(int) * nb, hipMemcpyDeviceToHost));
    used = std::min<int64_t>(int64_t(curh), capacity);
    std::vector<int> again;
    for (int b : todo)
      if (blkstat[b] & ST_DEFERRED) again.push_back(b);
    if (!again.empty()) {
      // grow the pool (keeping what is stored) and redo the deferred blocks
      int64_t newcap = capacity * 2;
      DevBuf bigger;
      GCQ_TRY(bigger.ensure(size_t(newcap) * csz + 256));
      GCQ_HIP(hipMemcpy(bigger.p, F.slices.p, size_t(used) * csz, hipMemcpyDeviceToDevice));
      std::swap(bigger.p, F.slices.p);
      std::swap(bigger.bytes, F.slices.bytes);
      capacity = newcap;
    }
    todo.swap(again);
  }
  if (!todo.empty()) return fail(GCQ_ERR_NOMEM, "3D-ACA pool could not hold the result");
  GCQ_HIP(hipMemcpy(terms.data(), d_terms, sizeof(Term3) * terms.size(), hipMemcpyDeviceToHost));
  ctx->kernel_ms["aca3d"] = ms;
  ctx->kernel_ms["aca3d_far"] = ms_far;
  ctx->kernel_ms["aca3d_near"] = ms_near;
  ctx->kernel_ms["aca3d_tensor"] = ms_tensor;
  ctx->kernel_ms["aca3d_rounds"] = rounds;
  // host tables
  F.brank.assign(blkrank.begin(), blkrank.end());
  F.bterm.assign(nb, 0);
  F.tfreq.clear();
  F.trank.clear();
  F.toff.clear();
  std::vector<int64_t> foff;
  int nt = 0;
  int ncap = 0;
  int64_t store = 0, slice_rank_sum = 0;
  for (int b = 0; b < nb; ++b) {
    F.bterm[b] = nt;
    ncap += (blkstat[b] & ST_CAPPED) != 0;
    for (int d = 0; d < F.brank[b]; ++d) {
      const Term3& t = terms[size_t(b) * R3_MAX + d];
      F.tfreq.push_back(t.freq);
      F.trank.push_back(t.rank);
      F.toff.push_back(t.slice);
      foff.push_back(t.fiber);
      store += (t.rank < 0 ? int64_t(bd[b].m) * bd[b].n : int64_t(t.rank) * (bd[b].m + bd[b].n)) + nK;
      if (t.rank >= 0) slice_rank_sum += t.rank;
      ++nt;
    }
  }
  F.bterm.push_back(nt);
  F.tfoff = foff;
  GCQ_TRY(upload(F.d_brank, F.brank, ctx->stream));
  GCQ_TRY(upload(F.d_bterm, F.bterm, ctx->stream));
  GCQ_TRY(upload(F.d_trank, F.trank, ctx->stream));
  GCQ_TRY(upload(F.d_toff, F.toff, ctx->stream));
  GCQ_TRY(upload(F.d_tfoff, F.tfoff, ctx->stream));
  {
    // product tables: stacked far columns and the block order of the product
    std::vector<int64_t> cols;
    std::vector<int32_t> bcol(nb + 1, 0);
    std::vector<double> work(nb, 0.0);
    for (int b = 0; b < nb; ++b) {
      bcol[b] = int32_t(cols.size() / 3);
      for (int d = 0; d < F.brank[b]; ++d) {
        const int ti = F.bterm[b] + d;
        if (F.trank[ti] < 0) {
          work[b] += double(bd[b].m) * bd[b].n;
          continue;
        }
        for (int c = 0; c < F.trank[ti]; ++c) {
          cols.push_back(F.toff[ti] + int64_t(c) * bd[b].m);                                    // Ubar col
          cols.push_back(F.toff[ti] + int64_t(F.trank[ti]) * bd[b].m + int64_t(c) * bd[b].n);   // Vbar col
          cols.push_back(F.tfoff[ti]);
          work[b] += bd[b].m + bd[b].n;
        }
      }
    }
    bcol[nb] = int32_t(cols.size() / 3);
    std::vector<int32_t> mo;
    for (int b = 0; b < nb; ++b)
      if (F.brank[b] > 0) mo.push_back(b);
    std::stable_sort(mo.begin(), mo.end(), [&](int a, int b) { return work[a] > work[b]; });
    F.n_mvblocks = int(mo.size());
    GCQ_TRY(upload(F.d_cols, cols, ctx->stream));
    GCQ_TRY(upload(F.d_bcol, bcol, ctx->stream));
    GCQ_TRY(upload(F.d_mvorder, mo, ctx->stream));
  }
  GCQ_HIP(hipStreamSynchronize(ctx->stream));
  F.storage_bytes = store * csz;
  F.dense_bytes = int64_t(ctx->n) * ctx->n * nK * csz;
  F.valid = true;
  if (stats) {
    std::memset(stats, 0, sizeof(*stats));
    stats->n_blocks = nb;
    int rmin = 1 << 30, rmx = 0;
    double rs = 0;
    for (int b = 0; b < nb; ++b) {
      rmin = std::min(rmin, F.brank[b]);
      rmx = std::max(rmx, F.brank[b]);
      rs += F.brank[b];
    }
    stats->rank_min = nb ? rmin : 0;
    stats->rank_max = rmx;
    stats->rank_mean = nb ? rs / nb : 0.0;
    stats->n_capped = ncap;
    stats->slice_rank_sum = slice_rank_sum;
    stats->storage_bytes = F.storage_bytes;
    stats->compression_rate = double(F.storage_bytes) / double(F.dense_bytes);
    stats->device_ms = ms;
  }
  return ncap > 0 ? GCQ_RANK_CAPPED : GCQ_OK;
}

extern "C" GCQ_API int gcq_get_aca3d_block(gcq_context* ctx, int32_t block, int32_t cap,
                                           int32_t* rank, int32_t* freqs, gcq_c128* fibers,
                                           gcq_c128* slices) {
  if (!ctx) return fail(GCQ_ERR_ARG, "ctx is NULL");
  if (!ctx->F.valid) return fail(GCQ_ERR_STATE, "run gcq_aca3d first");
  if (block < 0 || block >= int(ctx->blocks.size())) return fail(GCQ_ERR_ARG, "bad block");
  if (!rank) return fail(GCQ_ERR_ARG, "rank is NULL");
  const Faces3D& F = ctx->F;
  const int r = F.brank[block];
  *rank = r;
  if (r > cap) return fail(GCQ_ERR_ARG, "rank %d exceeds cap %d", r, cap);
  const Block& B = ctx->blocks[block];
  const int m = ctx->clusters[B.row].end - ctx->clusters[B.row].begin;
  const int n = ctx->clusters[B.col].end - ctx->clusters[B.col].begin;
  const int nK = F.nK;
  auto fetch = [&](int64_t off, int64_t cnt, std::vector<std::complex<double>>& out) -> int {
    out.resize(cnt);
    if (F.precision == GCQ_C128) {
      GCQ_HIP(hipMemcpy(out.data(), F.slices.as<cpx<double>>() + off, cnt * 16,
                        hipMemcpyDeviceToHost));
    } else {
      std::vector<cpx<float>> t(cnt);
      GCQ_HIP(hipMemcpy(t.data(), F.slices.as<cpx<float>>() + off, cnt * 8, hipMemcpyDeviceToHost));
      for (int64_t e = 0; e < cnt; ++e) out[e] = {t[e].re, t[e].im};
    }
    return GCQ_OK;
  };
  for (int d = 0; d < r; ++d) {
    const int ti = F.bterm[block] + d;
    if (freqs) freqs[d] = F.tfreq[ti];
    std::vector<std::complex<double>> buf;
    if (fibers) {
      GCQ_TRY(fetch(F.tfoff[ti], nK, buf));
      std::memcpy(fibers + int64_t(d) * nK, buf.data(), sizeof(gcq_c128) * nK);
    }
    if (slices) {
      gcq_c128* out = slices + int64_t(d) * m * n;
      if (F.trank[ti] < 0) {
        GCQ_TRY(fetch(F.toff[ti], int64_t(m) * n, buf));
        std::memcpy(out, buf.data(), sizeof(gcq_c128) * m * n);
      } else {
        const int t = F.trank[ti];
        GCQ_TRY(fetch(F.toff[ti], int64_t(t) * (m + n), buf));
        for (int j = 0; j < n; ++j)
          for (int i = 0; i < m; ++i) {
            std::complex<double> acc = 0;
            for (int c = 0; c < t; ++c)
              acc += buf[int64_t(c) * m + i] * std::conj(buf[int64_t(t) * m + int64_t(c) * n + j]);
            out[int64_t(j) * m + i] = {acc.real(), acc.imag()};
          }
      }
    }
  }
  return GCQ_OK;
}
