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

// LDS of the far kernel per group size NW (waves per block).  One area serves
// three uses that never overlap in time: the residual coefficients of the
// slice ACA (RES of them: the sum of the accepted slices' ranks; a block whose
// slices need more is redone by the next larger group), the recompression
// matrices (ranks up to JK in LDS, larger ones in the global workspace), the
// 16 KB row staging of the slice inner products and the factor staging of the
// pivot search (at most 24 KB).
template <int NW>
struct Cls;
template <>
struct Cls<1> {
  static constexpr int JK = 19;
};
template <>
struct Cls<2> {
  static constexpr int JK = 24;
};
template <>
struct Cls<4> {
  static constexpr int JK = 28;
};
template <>
struct Cls<8> {
  static constexpr int JK = 36;
};

enum : int {
  ST_ESCALATE = 32    // residual coefficients exceed the group's LDS capacity
};

template <typename T, int NW>
struct Shared3 {
  static constexpr int A0 = 3 * Cls<NW>::JK * Cls<NW>::JK * 16;
  static constexpr int A1 = A0 > 16384 ? A0 : 16384;
  // the largest group holds every possible stack (R3_MAX slices of rank <= 64)
  static constexpr int A2 = NW == 8 ? R3_MAX * 64 * int(sizeof(cpx<T>)) : 0;
  static constexpr int BYTES = A1 > A2 ? A1 : A2;
  static constexpr int RES0 = BYTES / int(sizeof(cpx<T>));
  static constexpr int RES = RES0 < R3_MAX * 64 ? RES0 : R3_MAX * 64;
  static constexpr int JK = Cls<NW>::JK;
  union {
    cpx<T> coef[RES0];          // residual coefficients of the current row / column
    cpx<double> mats[BYTES / 16];
  };
  AcaShared<T> aca;
  RecompShared rs;
  Term3 term[R3_MAX];
  unsigned char cterm[RES];    // slice of each stacked column
  cpx<T> fk[R3_MAX];           // f_d[k_cur]
  cpx<T> hp[R3_MAX];           // H_d[i_l, j_l]
  cpx<double> hin[R3_MAX];     // <H_d, H_l>
  cpx<double> colsum[64];      // per-column sums of the slice inner products
  unsigned usedk[NK_MAX / 32];
  int64_t alloc;
  int idx;
};

// pool allocation by one lane; returns -1 when the pool is exhausted
__device__ inline int64_t pool_alloc(unsigned long long* cursor, int64_t cnt, int64_t capacity) {
  unsigned long long o = atomicAdd(cursor, (unsigned long long)cnt);
  if (int64_t(o) + cnt > capacity) return -1;
  return int64_t(o);
}

// residual entry function of a far block at one frequency:
//   R(i, j) = A_ij(s) - sum_d f_d[k] (Ubar_d Vbar_d^H)[i, j]
// over the nres stacked columns x of the accepted slices (x of slice cterm[x]).
// A row (column) evaluation first forms the coefficients f_d[k] Ubar[i][x]
// (f_d[k] conj(Vbar[j][x])) in LDS; each entry then subtracts
// sum_x coef[x] conj(Vbar[j][x]) (sum_x Ubar[i][x] coef[x]).
template <typename T, bool ALLFAR, int NW, bool DLP>
struct ResidualEntry {
  const Tab* tab;
  int rb, cb, m, n;
  double sr, si;
  bool all_far;
  int nres;
  Shared3<T, NW>* sh;
  const cpx<T>* Us;   // stacked Ubar columns (m apart)
  const cpx<T>* Vs;   // stacked Vbar columns (n apart)
  bool rowmode;
  __device__ void prep_row(int i) {
    for (int x = threadIdx.x; x < nres; x += NW * WAVE)
      sh->coef[x] = cmul(sh->fk[sh->cterm[x]], Us[int64_t(x) * m + i]);
    rowmode = true;
    __syncthreads();
  }
  __device__ void prep_col(int j) {
    for (int x = threadIdx.x; x < nres; x += NW * WAVE) {
      const cpx<T> v = Vs[int64_t(x) * n + j];
      sh->coef[x] = cmul(sh->fk[sh->cterm[x]], cpx<T>{v.re, -v.im});
    }
    rowmode = false;
    __syncthreads();
  }
  // part p of P of the residual entry (i, j): quadrature points and stacked
  // columns x = p, p + P, ...
  __device__ cpx<T> part(int i, int j, int p, int P) const {
    cpx<T> a = op_entry_part<T, ALLFAR, DLP>(*tab, rb + i, cb + j, sr, si, all_far, p, P);
    T ar = 0, ai = 0;
    const cpx<T>* q = sh->coef;
    if (rowmode) {
      const cpx<T>* V = Vs + j;
#pragma unroll 12
      for (int x = p; x < nres; x += P) {
        const cpx<T> v = V[int64_t(x) * n], c = q[x];
        ar += c.re * v.re + c.im * v.im;   // c conj(v)
        ai += c.im * v.re - c.re * v.im;
      }
    } else {
      const cpx<T>* U = Us + i;
#pragma unroll 12
      for (int x = p; x < nres; x += P) {
        const cpx<T> u = U[int64_t(x) * m], c = q[x];
        ar += u.re * c.re - u.im * c.im;
        ai += u.re * c.im + u.im * c.re;
      }
    }
    a.re -= ar;
    a.im -= ai;
    return a;
  }
};

// entry (i, j) of a factored slice, sum_c Ubar[i][c] conj(Vbar[j][c]) (one thread)
template <typename T>
__device__ inline cpx<T> slice_at(const Term3& t, const cpx<T>* pool, int m, int n, int i, int j) {
  const cpx<T>* U = pool + t.slice;
  const cpx<T>* V = pool + t.vslice;
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
// first in row-major order on ties.  The product is expanded chunk by chunk
// (CR x CC entries, one 4 x 4 tile per thread) and never stored; the chunk's
// rows of Ubar and Vbar pass through LDS TC columns at a time, so that every
// factor entry is read once per chunk row / column instead of once per tile.
// stage: LDS scratch of (CR + CC) * 128 bytes.
template <typename T, int NW>
__device__ inline void lowrank_argmax(const cpx<T>* __restrict__ U, const cpx<T>* __restrict__ V,
                                      int m, int n, int t, double& best, int& be, cpx<T>* stage) {
  constexpr int NT = NW * WAVE;
  constexpr int CR = NW >= 4 ? 64 : 32;                  // chunk rows
  constexpr int CC = NT * 16 / CR;                       // chunk columns: NT tiles of 4 x 4
  constexpr int TC = int(128 / sizeof(cpx<T>));          // factor columns per stage
  const int tid = threadIdx.x;
  cpx<T>* su = stage;             // [c][r], CR rows
  cpx<T>* sv = stage + TC * CR;   // [c][j], CC rows
  const int ti = tid % (CR / 4), tj = tid / (CR / 4);    // this thread's tile in the chunk
  best = -1.0;
  be = 0x7fffffff;
  for (int i0 = 0; i0 < m; i0 += CR) {
    for (int j0 = 0; j0 < n; j0 += CC) {
      cpx<T> acc[4][4];
#pragma unroll
      for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y) acc[x][y] = {T(0), T(0)};
      for (int c0 = 0; c0 < t; c0 += TC) {
        __syncthreads();
        for (int e = tid; e < TC * CR; e += NT) {
          const int c = e / CR, r = e % CR;
          su[e] = (c0 + c < t && i0 + r < m) ? U[int64_t(c0 + c) * m + i0 + r] : cpx<T>{T(0), T(0)};
        }
        for (int e = tid; e < TC * CC; e += NT) {
          const int c = e / CC, r = e % CC;
          sv[e] = (c0 + c < t && j0 + r < n) ? V[int64_t(c0 + c) * n + j0 + r] : cpx<T>{T(0), T(0)};
        }
        __syncthreads();
        const int cn = min(TC, t - c0);
        for (int c = 0; c < cn; ++c) {
          cpx<T> u[4], v[4];
#pragma unroll
          for (int x = 0; x < 4; ++x) {
            u[x] = su[c * CR + 4 * ti + x];
            v[x] = sv[c * CC + 4 * tj + x];
          }
#pragma unroll
          for (int x = 0; x < 4; ++x)
#pragma unroll
            for (int y = 0; y < 4; ++y) {   // u conj(v)
              acc[x][y].re += u[x].re * v[y].re + u[x].im * v[y].im;
              acc[x][y].im += u[x].im * v[y].re - u[x].re * v[y].im;
            }
        }
      }
#pragma unroll
      for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y) {
          const int i = i0 + 4 * ti + x, j = j0 + 4 * tj + y;
          if (i < m && j < n) {
            const double val = mag2(acc[x][y]);
            const int e = i * n + j;
            if (val > best || (val == best && e < be)) { best = val; be = e; }
          }
        }
    }
  }
  __syncthreads();
  grp_argmax<NW>(best, be);
}

// <H_d, H_l>_F for every accepted slice d and the candidate slice l (d = l
// included), in one pass over the block's stacked factors.  With
// P = Ubar_l^H [Ubar_0 .. Ubar_l] and Q = [Vbar_0 .. Vbar_l]^H Vbar_l,
// <H_d, H_l> = sum over the columns b of slice d and a of slice l of
// P[a][b] Q[b][a].  Stack columns [0, nres) hold the accepted slices in term
// order, [nres, nres + t) the candidate.  Pairs (a, b) are taken b-major, up
// to 64 columns b and PAIRS pairs per pass; each thread accumulates both
// factors of its pairs over the rows, staged through LDS R rows at a time.
// The products are then summed per column b and, by thread d, over the
// columns of slice d.  Writes h[d] (d <= ell, h[ell] = |H_l|^2).
// stage: LDS scratch of 16 KB; colsum: 64 complex doubles of LDS.
template <typename T, int NW>
__device__ inline void stack_inner(const cpx<T>* __restrict__ Us, const cpx<T>* __restrict__ Vs,
                                   int m, int n, int nres, int t, int ell, const Term3* terms,
                                   int64_t sbase, cpx<T>* stage, cpx<double>* colsum,
                                   cpx<double>* h) {
  constexpr int NT = NW * WAVE;
  constexpr int R = int(128 / sizeof(cpx<T>));   // 16 (float) or 8 (double)
  constexpr int PAIRS = NT * 4 < 1024 ? NT * 4 : 1024;
  constexpr int PP = PAIRS / NT;
  const int tid = threadIdx.x;
  cpx<T>* sl = stage;           // [column][r]
  cpx<T>* sd = stage + 64 * R;  // [column][r]
  cpx<double>* prod = reinterpret_cast<cpx<double>*>(stage);   // after the row loops
  const int W = nres + t;
  const int nbmax = min(64, PAIRS / t);
  // the columns of this thread's slice d = tid
  int c_lo = 0, c_hi = 0;
  if (tid < ell) {
    c_lo = int((terms[tid].slice - sbase) / m);
    c_hi = c_lo + terms[tid].rank;
  } else if (tid == ell) {
    c_lo = nres;
    c_hi = W;
  }
  double hr = 0.0, hi = 0.0;
  const cpx<T>* Ul = Us + int64_t(nres) * m;
  const cpx<T>* Vl = Vs + int64_t(nres) * n;
  for (int b0 = 0; b0 < W; b0 += nbmax) {
    const int nb = min(nbmax, W - b0);
    const int npair = nb * t;
    double pr[PP], pi[PP], qr[PP], qi[PP];
    int pb[PP], pa[PP];
#pragma unroll
    for (int q = 0; q < PP; ++q) {
      pr[q] = pi[q] = qr[q] = qi[q] = 0.0;
      const int p = q * NT + tid;
      pb[q] = p / t;
      pa[q] = p % t;
    }
    for (int side = 0; side < 2; ++side) {
      const int len = side == 0 ? m : n;
      const cpx<T>* X = side == 0 ? Ul : Vs + int64_t(b0) * n;   // conjugated operand
      const cpx<T>* Y = side == 0 ? Us + int64_t(b0) * m : Vl;
      const int tx = side == 0 ? t : nb, ty = side == 0 ? nb : t;
      for (int r0 = 0; r0 < len; r0 += R) {
        const int rn = min(R, len - r0);
        __syncthreads();
        for (int e = tid; e < tx * R; e += NT) {
          const int c = e / R, r = e % R;
          sl[e] = r < rn ? X[int64_t(c) * len + r0 + r] : cpx<T>{T(0), T(0)};
        }
        for (int e = tid; e < ty * R; e += NT) {
          const int c = e / R, r = e % R;
          sd[e] = r < rn ? Y[int64_t(c) * len + r0 + r] : cpx<T>{T(0), T(0)};
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < PP; ++q) {
          if (q * NT + tid < npair) {
            const int ax = side == 0 ? pa[q] : pb[q], ay = side == 0 ? pb[q] : pa[q];
            double sr = 0.0, si = 0.0;
#pragma unroll 4
            for (int r = 0; r < R; ++r) {
              const cpx<T> x = sl[ax * R + r], y = sd[ay * R + r];
              sr += double(x.re) * y.re + double(x.im) * y.im;   // conj(x) y
              si += double(x.re) * y.im - double(x.im) * y.re;
            }
            if (side == 0) { pr[q] += sr; pi[q] += si; } else { qr[q] += sr; qi[q] += si; }
          }
        }
      }
    }
    __syncthreads();   // the staging area becomes the product array
#pragma unroll
    for (int q = 0; q < PP; ++q) {
      const int p = q * NT + tid;
      if (p < npair) prod[p] = {pr[q] * qr[q] - pi[q] * qi[q], pr[q] * qi[q] + pi[q] * qr[q]};
    }
    __syncthreads();
    if (tid < nb) {
      double sr = 0.0, si = 0.0;
      for (int a = 0; a < t; ++a) {
        const cpx<double> v = prod[tid * t + a];
        sr += v.re;
        si += v.im;
      }
      colsum[tid] = {sr, si};
    }
    __syncthreads();
    const int lo = max(c_lo, b0), hi2 = min(c_hi, b0 + nb);
    for (int c = lo; c < hi2; ++c) {
      hr += colsum[c - b0].re;
      hi += colsum[c - b0].im;
    }
  }
  if (tid <= ell) h[tid] = {hr, hi};
  __syncthreads();
}

// 3D-ACA of admissible blocks, NW waves per block.  ALLFAR = true: blocks
// without self/near-tier entries (the float64 quadrature tiers are not
// compiled in); ALLFAR = false: admissible blocks that contain some.
template <typename T, bool ALLFAR, int NW, bool DLP>
__global__ void __launch_bounds__(NW * 64) aca3d_kernel(
    Tab tab, const BlockDesc3* __restrict__ blocks, const int* __restrict__ order, int nblocks,
    const double2* __restrict__ sigK, int nK, double tol_aca, double tol, int rmax, int aca_cap,
    unsigned char* __restrict__ ws, int64_t ws_stride, cpx<T>* __restrict__ pool,
    unsigned long long* __restrict__ cursor, int64_t capacity, Term3* __restrict__ terms,
    int* __restrict__ brank, int* __restrict__ bstatus, int* __restrict__ counter,
    unsigned long long* __restrict__ work) {
  constexpr int NT = NW * WAVE;
  using SH = Shared3<T, NW>;
  constexpr int JK = SH::JK;
  __shared__ SH sh;
  const int tid = threadIdx.x;
  const int lane = tid & (WAVE - 1), wid = tid / WAVE;
  // per-group workspace: ACA factors and Gram matrices, Jacobi matrices of
  // ranks above JK, Gram matrix <H_d, H_d'> of the accepted slices
  unsigned char* myws = ws + int64_t(blockIdx.x) * ws_stride;
  for (;;) {
    if (tid == 0) sh.idx = atomicAdd(counter, 1);
    __syncthreads();
    const int idx = uni(sh.idx);
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
    cpx<double>* G3 = jmats + 4 * 64 * 64;
    for (int w = opaque_tid(); w < (nK + 31) / 32; w += NT) sh.usedk[w] = 0u;
    // the block's stacked slice factors: U (m x S) then V (n x S)
    int S = B.sres;
    if (tid == 0) sh.alloc = pool_alloc(cursor, int64_t(m + n) * S, capacity);
    __syncthreads();
    int64_t sbase = uni64(sh.alloc);
    int ell = 0, kcur = 0, status = 0, nres = 0;
    double norm2 = 0.0;
    // algorithmic work of this block: entries and operations (see gcq_aca3d_stats)
    // (integers of wave-uniform values, so that they stay in scalar registers)
    int64_t wentries = 0, wflops = 0;
    if (sbase < 0) status |= ST_DEFERRED;
    cpx<T>* Us = pool + (sbase < 0 ? 0 : sbase);
    cpx<T>* Vs = Us + int64_t(S) * m;
    while (sbase >= 0) {
      for (int d = tid; d < ell; d += NT) sh.fk[d] = pool[sh.term[d].fiber + kcur];
      __syncthreads();
      const double2 sg = sigK[kcur];
      // nu = |sum_d f_d[k] H_d|_F, the current approximation of the block at
      // k: the slice tolerance is taken relative to max(|residual|, nu)
      double nu2 = 0.0;
      for (int e = tid; e < ell * ell; e += NT) {
        const int d = e / ell, d2 = e % ell;
        const cpx<T> a = sh.fk[d], bb = sh.fk[d2];
        const cpx<double> g = G3[d * R3_MAX + d2];
        // a conj(b) <H_d, H_d2>
        const double pr = double(a.re) * bb.re + double(a.im) * bb.im;
        const double pi = double(a.im) * bb.re - double(a.re) * bb.im;
        nu2 += pr * g.re - pi * g.im;
      }
      const double nu = unid(sqrt(fmax(grp_sum<NW>(nu2), 0.0)));
      // ---- residual slice at k_cur: ACA, then recompression
      ResidualEntry<T, ALLFAR, NW, DLP> ent{&tab, B.rb, B.cb, m, n, sg.x, sg.y, B.all_far != 0, nres, &sh,
                                       Us, Vs, true};
      int ast = 0;
      const int k = uni(aca_grp<NW, true, T>(ent, m, n, cap, aca_cap, tol_aca, nu, U, W, GU, GV, sh.aca, ast));
      ast = uni(ast);
      if (ast & ST_CAPPED) status |= ST_CAPPED;
      {
        // rows (length n) and columns (length m) with their residual sums
        const int64_t e = int64_t(uni(sh.aca.nrows)) * n + int64_t(k) * m;
        wentries += e;
        // residual terms; Gram entries (8 (m + n) per pair, twice: k (k - 1) / 2 pairs)
        wflops += e * (7 * 20 + 8 * int64_t(nres)) + 12 * int64_t(m + n) * k * (k - 1);
      }
      // working matrices in LDS when they fit, else in the workspace (two call
      // sites, so that the LDS one compiles to LDS instructions)
      int t;
      if (recompress_mats(k) <= recompress_mats(JK))
        t = uni(recompress_grp<NW>(k, cap, GU, GV, tol_aca, nu, true, sh.mats, sh.rs));
      else
        t = uni(recompress_grp<NW>(k, cap, GU, GV, tol_aca, nu, true, jmats, sh.rs));
      // the candidate slice goes to the next free stacked columns
      if (nres + t > SH::RES) { status |= ST_ESCALATE; break; }   // needs a larger group
      if (nres + t > S) {
        // move the stack to a reservation twice as large (the old one is left unused)
        const int S2 = min(R3_MAX * 64, max(2 * S, ((nres + t + 15) / 16) * 16));
        if (tid == 0) sh.alloc = pool_alloc(cursor, int64_t(m + n) * S2, capacity);
        __syncthreads();
        const int64_t nbase = uni64(sh.alloc);
        if (nbase < 0) { status |= ST_DEFERRED; break; }
        cpx<T>* nUs = pool + nbase;
        cpx<T>* nVs = nUs + int64_t(S2) * m;
        for (int64_t e = tid; e < int64_t(nres) * m; e += NT) nUs[e] = Us[e];
        for (int64_t e = tid; e < int64_t(nres) * n; e += NT) nVs[e] = Vs[e];
        if (tid == 0) {
          for (int d = 0; d < ell; ++d) {
            const int64_t c0 = (sh.term[d].slice - sbase) / m;
            sh.term[d].slice = nbase + c0 * m;
            sh.term[d].vslice = nbase + int64_t(S2) * m + c0 * n;
          }
        }
        __syncthreads();
        sbase = nbase;
        S = S2;
        Us = nUs;
        Vs = nVs;
      }
      apply_factors<T>(k, t, m, n, U, W, GU, GV, Us + int64_t(nres) * m, Vs + int64_t(nres) * n, tid,
                       NT);
      __syncthreads();
      Term3 cur;
      cur.slice = sbase + int64_t(nres) * m;
      cur.vslice = sbase + int64_t(S) * m + int64_t(nres) * n;
      cur.rank = t;
      cur.freq = kcur;
      // ---- pivot: largest modulus, first in row-major order on ties
      wflops += 8 * (int64_t(t) * (m + n) * k + int64_t(m) * n * t);   // apply, expansion
      double best;
      int be;
      lowrank_argmax<T, NW>(pool + cur.slice, pool + cur.vslice, m, n, t, best, be,
                            reinterpret_cast<cpx<T>*>(sh.mats));
      if (!(best > PivFloor<T>::v)) break;   // zero pivot: rank stays ell
      be = uni(be);
      const int ip = be / n, jp = be % n;
      const cpx<T> piv = slice_at<T>(cur, pool, m, n, ip, jp);
      for (int d = tid; d < ell; d += NT) sh.hp[d] = slice_at<T>(sh.term[d], pool, m, n, ip, jp);
      if (tid == 0) sh.alloc = pool_alloc(cursor, nK, capacity);
      __syncthreads();
      const int64_t foff = uni64(sh.alloc);
      if (foff < 0) { status |= ST_DEFERRED; break; }
      cur.fiber = foff;
      // ---- fiber over K
      wentries += nK;
      wflops += int64_t(nK) * (7 * 20 + 8 * ell);
      {
        int tt = t;
        for (int d = 0; d < ell; ++d) tt += sh.term[d].rank;
        wflops += 8 * int64_t(t) * uni(tt) * (m + n) + 8 * int64_t(nK) * ell;   // inner products
      }
      const cpx<T> inv = cinv(piv);
      double nf2 = 0.0;
      for (int kk = tid; kk < nK; kk += NT) {
        const double2 s2 = sigK[kk];
        cpx<T> a;
        if constexpr (DLP)
          a = dlp_entry_part<T, ALLFAR>(tab, B.rb + ip, B.cb + jp, s2.x, s2.y, B.all_far != 0, 0, 1);
        else
          a = entry<T, ALLFAR>(tab, B.rb + ip, B.cb + jp, s2.x, s2.y, B.all_far != 0);
        for (int d = 0; d < ell; ++d) {
          cpx<T> p = cmul(sh.hp[d], pool[sh.term[d].fiber + kk]);
          a.re -= p.re;
          a.im -= p.im;
        }
        cpx<T> f = cmul(a, inv);
        pool[foff + kk] = f;
        nf2 += double(f.re) * double(f.re) + double(f.im) * double(f.im);
      }
      __syncthreads();
      nf2 = unid(grp_sum<NW>(nf2));
      // ---- eq. norm: <H_d, H_l> = tr((U_l^H U_d)(V_d^H V_l)), |H_l|^2 with d = l
      stack_inner<T, NW>(Us, Vs, m, n, nres, t, ell, sh.term, sbase, reinterpret_cast<cpx<T>*>(sh.mats),
                         sh.colsum, sh.hin);
      const double nh2 = unid(sh.hin[ell].re);
      // <f_d, f_l> = sum f_d conj(f_l), slice d by wave d mod NW
      double crossw = 0.0;
      for (int d = wid; d < ell; d += NW) {
        double fr = 0, fi = 0;
        for (int kk = lane; kk < nK; kk += WAVE) {
          cpx<T> x = pool[sh.term[d].fiber + kk], y = pool[foff + kk];
          fr += double(x.re) * y.re + double(x.im) * y.im;
          fi += double(x.im) * y.re - double(x.re) * y.im;
        }
        fr = wave_sum(fr);
        fi = wave_sum(fi);
        crossw += sh.hin[d].re * fr - sh.hin[d].im * fi;
      }
      const double cross = unid(grp_sum<NW>(lane == 0 ? crossw : 0.0));
      norm2 += 2.0 * cross + nh2 * nf2;
      if (tid == 0) sh.usedk[kcur >> 5] |= 1u << (kcur & 31);
      __syncthreads();
      if (sqrt(fmax(nh2 * nf2, 0.0)) <= tol * sqrt(fmax(norm2, 0.0))) break;  // drop term l
      if (tid == 0) sh.term[ell] = cur;
      for (int x = tid; x < t; x += NT) sh.cterm[nres + x] = (unsigned char)ell;
      nres += t;
      for (int d = opaque_tid(); d <= ell; d += NT) {
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
      for (int kk = opaque_tid(); kk < nK; kk += NT) {
        if ((sh.usedk[kk >> 5] >> (kk & 31)) & 1u) continue;
        double v = mag2(pool[foff + kk]);
        if (v > bf) { bf = v; bk = kk; }
      }
      grp_argmax<NW>(bf, bk);
      bk = uni(bk);
      bf = unid(bf);
      if (bk == 0x7fffffff) break;                       // every frequency used
      if (ell >= rmax) { status |= ST_CAPPED; break; }
      if (!(bf > 0.0)) break;                            // fiber zero at all unused ones
      kcur = bk;
    }
    __syncthreads();
    for (int d = opaque_tid(); d < ell; d += NT) terms[int64_t(b) * R3_MAX + d] = sh.term[d];
    if (tid == 0) {
      brank[b] = ell;
      bstatus[b] = status;
      if (!(status & (ST_DEFERRED | ST_ESCALATE))) {
        atomicAdd(work, (unsigned long long)wentries);
        atomicAdd(work + 1, (unsigned long long)wflops);
      }
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
        t.vslice = -1;
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

// the accepted terms of every block, compacted: out[tb[b] + d] = terms[b R3_MAX + d]
static __global__ void gather_terms(const Term3* __restrict__ terms, const int* __restrict__ brank,
                                    const int* __restrict__ tb, int nb, Term3* __restrict__ out) {
  for (int b = blockIdx.x; b < nb; b += gridDim.x)
    for (int d = threadIdx.x; d < brank[b]; d += blockDim.x)
      out[tb[b] + d] = terms[int64_t(b) * R3_MAX + d];
}

// product table of the stacked far columns: column x of block b's stack
// (b's far terms in order, bcol[b] the first) gets its Ubar column, Vbar
// column and fiber offsets
static __global__ void build_cols(const int* __restrict__ blk, const int* __restrict__ bterm,
                                  const int* __restrict__ trank, const int64_t* __restrict__ toff,
                                  const int64_t* __restrict__ tvoff, const int64_t* __restrict__ tfoff,
                                  const int* __restrict__ bcol, int nb, int64_t* __restrict__ cols) {
  for (int b = blockIdx.x; b < nb; b += gridDim.x) {
    const int m = blk[5 * b + 1] - blk[5 * b], n = blk[5 * b + 3] - blk[5 * b + 2];
    int64_t c = bcol[b];
    for (int d = bterm[b]; d < bterm[b + 1]; ++d) {
      const int r = trank[d];
      if (r < 0) continue;   // dense slice of an inadmissible block
      for (int x = threadIdx.x; x < r; x += blockDim.x) {
        cols[3 * (c + x)] = toff[d] + int64_t(x) * m;
        cols[3 * (c + x) + 1] = tvoff[d] + int64_t(x) * n;
        cols[3 * (c + x) + 2] = tfoff[d];
      }
      c += r;
    }
  }
}

// launch of the far kernel with NW waves per block, single or double layer
template <typename T, bool AF, bool DLP, typename... Args>
static void launch_far_op(int nw, int grid, hipStream_t st, Args... args) {
  switch (nw) {
    case 1: hipLaunchKernelGGL((aca3d_kernel<T, AF, 1, DLP>), dim3(grid), dim3(64), 0, st, args...); break;
    case 2: hipLaunchKernelGGL((aca3d_kernel<T, AF, 2, DLP>), dim3(grid), dim3(128), 0, st, args...); break;
    case 4: hipLaunchKernelGGL((aca3d_kernel<T, AF, 4, DLP>), dim3(grid), dim3(256), 0, st, args...); break;
    default: hipLaunchKernelGGL((aca3d_kernel<T, AF, 8, DLP>), dim3(grid), dim3(512), 0, st, args...); break;
  }
}
template <typename T, bool AF, typename... Args>
static void launch_far(bool dlp, int nw, int grid, hipStream_t st, Args... args) {
  if (dlp)
    launch_far_op<T, AF, true>(nw, grid, st, args...);
  else
    launch_far_op<T, AF, false>(nw, grid, st, args...);
}

// dense near-field tensor of the blocks [q0, q1): far-tier entries, then self/near-tier ones
template <typename T, bool DLP>
static void launch_near3(gcq_context* ctx, dim3 g1, dim3 g2, int q0, int q1, int64_t base0, int64_t s0,
                         int64_t s1, int nK, cpx<T>* out, int64_t span) {
  hipLaunchKernelGGL((near_far_tier<T, DLP>), g1, dim3(256), 0, ctx->stream, ctx->tab(), ctx->d_blk.as<int>(),
                     ctx->d_near_ids.as<int>(), ctx->d_near_off.as<int64_t>(), q0, q1, base0,
                     ctx->scratchC.as<double2>(), nK, out, span);
  hipLaunchKernelGGL((near_sing<T, DLP>), g2, dim3(256), 0, ctx->stream, ctx->tab(), ctx->d_sing.as<SingEntry>(),
                     s0, s1, base0, ctx->scratchC.as<double2>(), nK, out, span);
}

// side streams and fork/join events of the context, created on first use
int ensure_side_streams(gcq_context* ctx) {
  if (!ctx->evfork) GCQ_HIP(hipEventCreateWithFlags(&ctx->evfork, hipEventDisableTiming));
  for (int i = 0; i < 3; ++i) {
    if (!ctx->side[i]) GCQ_HIP(hipStreamCreateWithFlags(&ctx->side[i], hipStreamNonBlocking));
    if (!ctx->evjoin[i]) GCQ_HIP(hipEventCreateWithFlags(&ctx->evjoin[i], hipEventDisableTiming));
  }
  return GCQ_OK;
}

// Alg. 1 with dense slices on a batch of precomputed tensors: block b =
// ids[qlist[i]] with descriptor desc[b] (m x n), its tensor at
// Cn[k * stride + off[qlist[i]] - base0 + e], terms into terms[b * R3_MAX + d]
void launch_dense_aca3d(int precision, int grid, hipStream_t st, const BlockDesc3* desc, const int* qlist,
                        int nq, const int* ids, const int64_t* off, int64_t base0, const void* Cn,
                        int64_t stride, int nK, double tol, int rmax, void* pool, unsigned long long* cursor,
                        int64_t capacity, Term3* terms, int* brank, int* bstatus, int* counter) {
  if (precision == GCQ_C128)
    hipLaunchKernelGGL(aca3d_near_kernel<double>, dim3(grid), dim3(64), 0, st, desc, qlist, nq, ids, off, base0,
                       static_cast<const cpx<double>*>(Cn), stride, nK, tol, rmax, static_cast<cpx<double>*>(pool),
                       cursor, capacity, terms, brank, bstatus, counter);
  else
    hipLaunchKernelGGL(aca3d_near_kernel<float>, dim3(grid), dim3(64), 0, st, desc, qlist, nq, ids, off, base0,
                       static_cast<const cpx<float>*>(Cn), stride, nK, tol, rmax, static_cast<cpx<float>*>(pool),
                       cursor, capacity, terms, brank, bstatus, counter);
}

}  // namespace gcq

using namespace gcq;

extern "C" GCQ_API int gcq_aca3d(gcq_context* ctx, double tol_aca, double tol,
                                 int32_t max_freq_rank, int32_t precision, uint32_t flags,
                                 gcq_aca3d_stats* stats) {
  return gcq::aca3d_run(ctx, tol_aca, tol, max_freq_rank, precision, flags & GCQ_FLAG_DOUBLE_LAYER, false, stats);
}

namespace gcq {

// the 3D-ACA of the partition; near_only: admissible blocks get no terms
// (the FMM-based variant compresses their M2L operators instead)
int aca3d_run(gcq_context* ctx, double tol_aca, double tol, int32_t max_freq_rank, int32_t precision,
              uint32_t flags, bool near_only, gcq_aca3d_stats* stats) {
  const bool dlp = (flags & GCQ_FLAG_DOUBLE_LAYER) != 0;
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
  F.drop_product_state();   // graphs and tables refer to the operator rebuilt below
  F.precision = precision;
  F.dlp = dlp;
  F.nK = nK;
  F.near_only = near_only;
  const int nb = int(ctx->blocks.size());
  std::vector<BlockDesc3> bd(nb);
  int maxm = 0, maxmn = 0;
  for (int b = 0; b < nb; ++b) {
    const Block& B = ctx->blocks[b];
    const Cluster& A = ctx->clusters[B.row];
    const Cluster& C = ctx->clusters[B.col];
    bd[b] = {A.begin, A.end - A.begin, C.begin, C.end - C.begin, B.admissible ? 1 : 0,
             B.all_far ? 1 : 0, 0, 0};
    if (B.admissible) {
      // stacked slice columns: room for a few slices of full ACA rank to start with
      const int r0 = std::min(std::min(bd[b].m, bd[b].n), 64);
      bd[b].sres = std::min(R3_MAX * 64, ((ctx->tune.aca3d_stack_slices * r0 + 15) / 16) * 16);
    }
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
  // per-group workspace: ACA factors + Gram matrices, Jacobi matrices, <H_d, H_d'>
  auto ws_stride_for = [&](int mn) -> int64_t {
    return ((precision == GCQ_C128 ? ws_bytes<double>(aca_cap, mn, 0) : ws_bytes<float>(aca_cap, mn, 0)) +
            int64_t(4) * 64 * 64 * 16 + int64_t(R3_MAX) * R3_MAX * 16 + 4095) & ~int64_t(4095);
  };
  const int cus = ctx->cus;
  GCQ_TRY(ensure_side_streams(ctx));
  // waves per admissible block, by size class (tuning table); doubled for a
  // block whose residual stack outgrows its group
  std::vector<int> bnw(nb, 1);
  for (int b = 0; b < nb; ++b) {
    if (!bd[b].admissible) continue;
    const int sz = bd[b].m + bd[b].n;
    const int c = sz <= 160 ? 0 : sz <= 320 ? 1 : sz <= 640 ? 2 : 3;
    bnw[b] = ctx->tune.aca3d_waves[c];
  }
  // pool: dense near slices and factored far slices, bump-allocated
  size_t freeb = 0, totalb = 0;
  GCQ_HIP(hipMemGetInfo(&freeb, &totalb));
  int64_t near_elems = 0, far_stack = 0;
  for (int b = 0; b < nb; ++b)
    if (bd[b].admissible) far_stack += near_only ? 0 : int64_t(bd[b].m + bd[b].n) * bd[b].sres;
    else near_elems += int64_t(bd[b].m) * bd[b].n;
  // expected need: dense slices (near) of ~max_freq_rank/2 terms each, the far
  // blocks' stack reservations, plus one fiber per term
  const int64_t rexp = std::max(8, int(max_freq_rank) / 2 + 4);
  int64_t want = near_elems * rexp + far_stack + int64_t(nb) * rexp * nK;
  // at most a quarter of the free memory, and after a first call on this
  // tree a quarter more than that call used (the pool grows between rounds
  // when a block's slices do not fit, so a short estimate costs a round)
  int64_t capacity = std::min<int64_t>(want, int64_t(double(freeb) * 0.25) / csz);
  if (F.last_used > 0 && F.last_nb == nb) capacity = std::min(capacity, F.last_used + F.last_used / 4 + (int64_t(1) << 20));
  // the pool of an earlier call is reused (its contents are rebuilt); it only
  // grows when this operator needs more
  GCQ_TRY(F.slices.ensure(size_t(capacity) * csz + 256));
  capacity = std::max<int64_t>(capacity, int64_t((F.slices.bytes - 256) / csz));
  std::vector<int32_t> blkrank(nb), blkstat(nb);
  std::vector<Term3> terms;
  GCQ_TRY(upload(ctx->scratchB, bd, ctx->stream));
  GCQ_TRY(upload(ctx->scratchC, sig, ctx->stream));
  // scratch layout: cursor (8 B), 16 work counters, terms, ranks, status, work order
  GCQ_TRY(ctx->scratchD.ensure(128 + sizeof(Term3) * size_t(nb) * R3_MAX + sizeof(int) * 3 * size_t(nb)));
  unsigned long long* d_cursor = ctx->scratchD.as<unsigned long long>();
  int* d_counter = reinterpret_cast<int*>(ctx->scratchD.as<unsigned char>() + 16);
  int* d_near_counter = d_counter + 8;
  unsigned long long* d_work = reinterpret_cast<unsigned long long*>(ctx->scratchD.as<unsigned char>() + 96);
  Term3* d_terms = reinterpret_cast<Term3*>(ctx->scratchD.as<unsigned char>() + 128);
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
  const std::vector<int64_t>& sing_off = ctx->sing_off;
  DevBuf& tensor = ctx->scratchT;
  const int64_t tensor_budget = std::max<int64_t>(int64_t(1) << 28,
                                                  std::min<int64_t>(int64_t(16) << 30, int64_t(double(freeb) * 0.15)));
  hipLaunchKernelGGL(zero_int_3d, dim3(1), dim3(64), 0, ctx->stream, reinterpret_cast<int*>(d_work), 4);
  // the dense near-field entries at every frequency of K, as the per-frequency
  // H-matrix of the same frequencies and precision holds them ([k][near
  // storage]), are reused instead of evaluated again
  const bool reuse_near = ctx->H.valid && ctx->H.dlp == dlp && ctx->H.precision == precision && ctx->H.freqs == ctx->K &&
                          ctx->H.near_slot_elems == ctx->near_total && ctx->H.near.p != nullptr;
  std::vector<int> opos(nb);
  for (int i = 0; i < nb; ++i) opos[order[i]] = i;
  std::vector<int> todo;
  for (int b : order)
    if (!(near_only && bd[b].admissible)) todo.push_back(b);
  // blocks left out keep rank 0
  hipLaunchKernelGGL(zero_int_3d, dim3((2 * nb + 63) / 64), dim3(64), 0, ctx->stream, d_rank, 2 * nb);
  for (int round = 0; round < 8 && !todo.empty(); ++round) {
    hipLaunchKernelGGL(zero_int_3d, dim3(1), dim3(64), 0, ctx->stream, d_counter, 16);
    unsigned long long cur0 = (unsigned long long)used;
    GCQ_HIP(hipMemcpyAsync(d_cursor, &cur0, sizeof(cur0), hipMemcpyHostToDevice, ctx->stream));
    // admissible blocks by group size (8, 4, 2, 1 waves) and kind (no
    // near-tier entries / some), then inadmissible blocks (from their entry
    // tensor); each list keeps the cost order
    std::vector<int> lists[8], lq;
    auto slot_of = [](int nw, bool allfar) {
      const int c = nw == 8 ? 0 : nw == 4 ? 1 : nw == 2 ? 2 : 3;
      return 2 * c + (allfar ? 0 : 1);
    };
    for (int b : todo) {
      if (bd[b].admissible) lists[slot_of(bnw[b], bd[b].all_far != 0)].push_back(b);
      else lq.push_back(near_pos[b]);
    }
    std::sort(lq.begin(), lq.end());
    std::vector<int> both;
    int loff[8], lgrid[8];
    int64_t lws[8], lstride[8], ws_total = 0;
    for (int l = 0; l < 8; ++l) {
      loff[l] = int(both.size());
      both.insert(both.end(), lists[l].begin(), lists[l].end());
      const int nw = 8 >> (l / 2);
      int mn = 0;
      for (int b : lists[l]) mn = std::max(mn, bd[b].m + bd[b].n);
      lgrid[l] = std::min<int>(int(lists[l].size()), cus * std::max(1, 8 / nw));
      lstride[l] = ws_stride_for(std::max(mn, 1));
      lws[l] = ws_total;
      ws_total += lstride[l] * lgrid[l];
    }
    const int nfar = int(both.size());
    both.insert(both.end(), lq.begin(), lq.end());
    GCQ_TRY(ctx->scratchA.ensure(size_t(std::max<int64_t>(ws_total, 1))));
    GCQ_HIP(hipMemcpyAsync(d_order, both.data(), sizeof(int) * both.size(), hipMemcpyHostToDevice,
                           ctx->stream));
    GCQ_TRY(timed_begin(ctx));
    // group sizes 8, 4, 2 on the side streams, 1 on the context stream, all
    // at once: the large blocks start together with the many small ones
    GCQ_HIP(hipEventRecord(ctx->evfork, ctx->stream));
    for (int i = 0; i < 3; ++i) GCQ_HIP(hipStreamWaitEvent(ctx->side[i], ctx->evfork, 0));
    for (int l = 0; l < 8; ++l) {
      const int cnt = int(lists[l].size());
      if (cnt == 0) continue;
      const int nw = 8 >> (l / 2);
      hipStream_t st = l / 2 < 3 ? ctx->side[l / 2] : ctx->stream;
      unsigned char* wsp = ctx->scratchA.as<unsigned char>() + lws[l];
      const bool af = (l % 2) == 0;
      if (precision == GCQ_C128) {
        auto go = [&](auto tag) {
          launch_far<double, decltype(tag)::value>(
              dlp, nw, lgrid[l], st, ctx->tab(), (const BlockDesc3*)ctx->scratchB.as<BlockDesc3>(),
              (const int*)(d_order + loff[l]), cnt, (const double2*)ctx->scratchC.as<double2>(), nK,
              tol_aca, tol, int(max_freq_rank), aca_cap, wsp, lstride[l], F.slices.as<cpx<double>>(),
              d_cursor, capacity, d_terms, d_rank, d_stat, d_counter + l, d_work);
        };
        if (af) go(std::true_type()); else go(std::false_type());
      } else {
        auto go = [&](auto tag) {
          launch_far<float, decltype(tag)::value>(
              dlp, nw, lgrid[l], st, ctx->tab(), (const BlockDesc3*)ctx->scratchB.as<BlockDesc3>(),
              (const int*)(d_order + loff[l]), cnt, (const double2*)ctx->scratchC.as<double2>(), nK,
              tol_aca, tol, int(max_freq_rank), aca_cap, wsp, lstride[l], F.slices.as<cpx<float>>(),
              d_cursor, capacity, d_terms, d_rank, d_stat, d_counter + l, d_work);
        };
        if (af) go(std::true_type()); else go(std::false_type());
      }
      GCQ_HIP(hipGetLastError());
    }
    for (int i = 0; i < 3; ++i) {
      GCQ_HIP(hipEventRecord(ctx->evjoin[i], ctx->side[i]));
      GCQ_HIP(hipStreamWaitEvent(ctx->stream, ctx->evjoin[i], 0));
    }
    ms_far += timed_end(ctx, "aca3d_far_round");
    // inadmissible blocks in batches whose entry tensor fits the budget
    size_t pos = 0;
    const int* d_q = d_order + nfar;
    while (pos < lq.size()) {
      size_t end = lq.size();
      int64_t base0 = 0, span = ctx->near_total;
      const void* tens = ctx->H.near.p;
      hipLaunchKernelGGL(zero_int_3d, dim3(1), dim3(64), 0, ctx->stream, d_near_counter, 1);
      if (!reuse_near) {
        const int q0 = lq[pos];
        end = pos;
        while (end < lq.size() &&
               (ctx->near_off[lq[end]] + int64_t(bd[ctx->near_ids[lq[end]]].m) * bd[ctx->near_ids[lq[end]]].n -
                ctx->near_off[q0]) * nK * csz <= tensor_budget)
          ++end;
        if (end == pos) end = pos + 1;
        const int q1 = lq[end - 1] + 1;
        base0 = ctx->near_off[q0];
        span = (q1 < int(ctx->near_off.size()) ? ctx->near_off[q1] : ctx->near_total) - base0;
        GCQ_TRY(tensor.ensure(size_t(span) * nK * csz + 256));
        // self/near-tier entries of [q0, q1)
        const int64_t s0 = int64_t(std::lower_bound(sing_off.begin(), sing_off.end(), base0) - sing_off.begin());
        const int64_t s1 = int64_t(std::lower_bound(sing_off.begin(), sing_off.end(), base0 + span) - sing_off.begin());
        GCQ_TRY(timed_begin(ctx));
        const dim3 g1(std::min(q1 - q0, 65536)), g2(4096);
        if (precision == GCQ_C128) {
          if (dlp)
            launch_near3<double, true>(ctx, g1, g2, q0, q1, base0, s0, s1, nK, tensor.as<cpx<double>>(), span);
          else
            launch_near3<double, false>(ctx, g1, g2, q0, q1, base0, s0, s1, nK, tensor.as<cpx<double>>(), span);
        } else {
          if (dlp)
            launch_near3<float, true>(ctx, g1, g2, q0, q1, base0, s0, s1, nK, tensor.as<cpx<float>>(), span);
          else
            launch_near3<float, false>(ctx, g1, g2, q0, q1, base0, s0, s1, nK, tensor.as<cpx<float>>(), span);
        }
        GCQ_HIP(hipGetLastError());
        ms_tensor += timed_end(ctx, "aca3d_tensor_batch");
        tens = tensor.p;
      }
      GCQ_TRY(timed_begin(ctx));
      const int cnt = int(end - pos);
      if (precision == GCQ_C128)
        hipLaunchKernelGGL(aca3d_near_kernel<double>, dim3(std::min(cnt, cus * 16)), dim3(64), 0,
                           ctx->stream, ctx->scratchB.as<BlockDesc3>(), d_q + pos, cnt,
                           ctx->d_near_ids.as<int>(), ctx->d_near_off.as<int64_t>(), base0,
                           static_cast<const cpx<double>*>(tens), span, nK, tol, int(max_freq_rank),
                           F.slices.as<cpx<double>>(), d_cursor, capacity, d_terms, d_rank,
                           d_stat, d_near_counter);
      else
        hipLaunchKernelGGL(aca3d_near_kernel<float>, dim3(std::min(cnt, cus * 16)), dim3(64), 0,
                           ctx->stream, ctx->scratchB.as<BlockDesc3>(), d_q + pos, cnt,
                           ctx->d_near_ids.as<int>(), ctx->d_near_off.as<int64_t>(), base0,
                           static_cast<const cpx<float>*>(tens), span, nK, tol, int(max_freq_rank),
                           F.slices.as<cpx<float>>(), d_cursor, capacity, d_terms, d_rank,
                           d_stat, d_near_counter);
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
    bool grow = false;
    for (int b : todo) {
      if (blkstat[b] & ST_DEFERRED) {
        again.push_back(b);
        grow = true;
      } else if (blkstat[b] & ST_ESCALATE) {
        again.push_back(b);
        bnw[b] = std::min(8, 2 * bnw[b]);
      }
    }
    std::sort(again.begin(), again.end(), [&](int x, int y) { return opos[x] < opos[y]; });  // cost order
    if (grow) {
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
  // download the accepted terms only (compacted on the device)
  std::vector<int32_t> tb(nb + 1, 0);
  for (int b = 0; b < nb; ++b) tb[b + 1] = tb[b] + blkrank[b];
  {
    DevBuf d_tb, d_compact;
    GCQ_TRY(upload(d_tb, tb, ctx->stream));
    GCQ_TRY(d_compact.ensure(sizeof(Term3) * size_t(std::max(tb[nb], 1))));
    hipLaunchKernelGGL(gather_terms, dim3(std::min(nb, 65536)), dim3(64), 0, ctx->stream, d_terms, d_rank,
                       d_tb.as<int>(), nb, d_compact.as<Term3>());
    GCQ_HIP(hipGetLastError());
    terms.resize(size_t(tb[nb]));
    GCQ_HIP(hipMemcpyAsync(terms.data(), d_compact.p, sizeof(Term3) * terms.size(), hipMemcpyDeviceToHost,
                           ctx->stream));
    GCQ_HIP(hipStreamSynchronize(ctx->stream));
  }
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
  F.tvoff.clear();
  std::vector<int64_t> foff;
  int nt = 0;
  int ncap = 0;
  int64_t store = 0, slice_rank_sum = 0;
  for (int b = 0; b < nb; ++b) {
    F.bterm[b] = nt;
    ncap += (blkstat[b] & ST_CAPPED) != 0;
    for (int d = 0; d < F.brank[b]; ++d) {
      const Term3& t = terms[size_t(tb[b]) + d];
      F.tfreq.push_back(t.freq);
      F.trank.push_back(t.rank);
      F.toff.push_back(t.slice);
      F.tvoff.push_back(t.vslice);
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
  GCQ_TRY(upload(F.d_tvoff, F.tvoff, ctx->stream));
  GCQ_TRY(upload(F.d_tfoff, F.tfoff, ctx->stream));
  {
    // product tables: stacked far columns (built on the device) and the block
    // order of the product
    std::vector<int32_t> bcol(nb + 1, 0);
    std::vector<double> work(nb, 0.0);
    for (int b = 0; b < nb; ++b) {
      int cnt = 0;
      int64_t nextu = -1, nextv = -1;
      for (int d = 0; d < F.brank[b]; ++d) {
        const int ti = F.bterm[b] + d;
        if (F.trank[ti] < 0) {
          work[b] += double(bd[b].m) * bd[b].n;
          continue;
        }
        // the product reads a far block's stacked columns as one m x R and one n x R matrix
        if (nextu >= 0 && (F.toff[ti] != nextu || F.tvoff[ti] != nextv))
          return fail(GCQ_ERR_STATE, "block %d: slice factors are not stacked", b);
        nextu = F.toff[ti] + int64_t(F.trank[ti]) * bd[b].m;
        nextv = F.tvoff[ti] + int64_t(F.trank[ti]) * bd[b].n;
        cnt += F.trank[ti];
        work[b] += double(F.trank[ti]) * (bd[b].m + bd[b].n);
      }
      bcol[b + 1] = bcol[b] + cnt;
    }
    std::vector<int32_t> mo;
    for (int b = 0; b < nb; ++b)
      if (F.brank[b] > 0) mo.push_back(b);
    std::stable_sort(mo.begin(), mo.end(), [&](int a, int b) { return work[a] > work[b]; });
    F.n_mvblocks = int(mo.size());
    GCQ_TRY(upload(F.d_bcol, bcol, ctx->stream));
    GCQ_TRY(upload(F.d_mvorder, mo, ctx->stream));
    GCQ_TRY(F.d_cols.ensure(sizeof(int64_t) * 3 * size_t(std::max(bcol[nb], 1))));
    hipLaunchKernelGGL(build_cols, dim3(std::min(nb, 65536)), dim3(64), 0, ctx->stream, ctx->d_blk.as<int>(),
                       F.d_bterm.as<int>(), F.d_trank.as<int>(), F.d_toff.as<int64_t>(),
                       F.d_tvoff.as<int64_t>(), F.d_tfoff.as<int64_t>(), F.d_bcol.as<int>(), nb,
                       F.d_cols.as<int64_t>());
    GCQ_HIP(hipGetLastError());
  }
  GCQ_HIP(hipStreamSynchronize(ctx->stream));
  F.storage_bytes = store * csz;
  F.dense_bytes = int64_t(ctx->n) * ctx->n * nK * csz;
  F.last_used = used;
  F.last_nb = nb;
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
    unsigned long long work[2] = {0, 0};
    GCQ_HIP(hipMemcpy(work, d_work, sizeof(work), hipMemcpyDeviceToHost));
    stats->far_entries = int64_t(work[0]);
    stats->far_flops = double(work[1]);
    stats->far_ms = ms_far;
  }
  return ncap > 0 ? GCQ_RANK_CAPPED : GCQ_OK;
}

}  // namespace gcq

extern "C" GCQ_API int gcq_aca3d_ranks(gcq_context* ctx, int32_t* terms, int32_t* columns, int64_t n) {
  if (!ctx) return fail(GCQ_ERR_ARG, "ctx is NULL");
  if (!ctx->F.valid) return fail(GCQ_ERR_STATE, "run gcq_aca3d first");
  const Faces3D& F = ctx->F;
  const int64_t nb = int64_t(ctx->blocks.size());
  if (!terms || !columns || n != nb) return fail(GCQ_ERR_ARG, "terms and columns must hold %lld values", (long long)nb);
  for (int64_t b = 0; b < nb; ++b) {
    terms[b] = F.brank[b];
    int c = 0;
    for (int d = F.bterm[b]; d < F.bterm[b + 1]; ++d) c += F.trank[d] > 0 ? F.trank[d] : 0;
    columns[b] = c;
  }
  return GCQ_OK;
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
        std::vector<std::complex<double>> vbuf;
        GCQ_TRY(fetch(F.toff[ti], int64_t(t) * m, buf));
        GCQ_TRY(fetch(F.tvoff[ti], int64_t(t) * n, vbuf));
        for (int j = 0; j < n; ++j)
          for (int i = 0; i < m; ++i) {
            std::complex<double> acc = 0;
            for (int c = 0; c < t; ++c)
              acc += buf[int64_t(c) * m + i] * std::conj(vbuf[int64_t(c) * n + j]);
            out[int64_t(j) * m + i] = {acc.real(), acc.imag()};
          }
      }
    }
  }
  return GCQ_OK;
}
