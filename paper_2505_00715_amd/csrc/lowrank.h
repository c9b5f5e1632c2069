// Wave-level routines for the low-rank face of Sec. 4, shared by the per-
// frequency ACA kernels and the 3D-ACA kernel.
//
// aca_wave: partially pivoted ACA of an entry function (one wave64).
// recompress_wave: QR/SVD recompression of the ACA factors, carried out
//   through their Gram matrices: with G_V = V^H V = Q L Q^H and
//   B = L^{1/2} Q^H G_U Q L^{1/2} = Z S^2 Z^H, the truncated SVD of U V^H is
//   (U Q L^{1/2} Z_t)(V Q L^{-1/2} Z_t)^H, because R_V = L^{1/2} Q^H satisfies
//   R_V^H R_V = G_V (it plays the role of the triangular QR factor) and
//   B = M^H M for the core M = R_U R_V^H.
// apply_factors: forms the recompressed factors from the coefficients.
#pragma once
#include "device_common.h"

namespace gcq {

constexpr int ACA_MAXM = 16384;  // rows per block handled by the ACA routine

struct PairDesc {
  int rb, m, cb, n;   // internal positions: rows [rb, rb+m), columns [cb, cb+n)
  int all_far;        // 1: no self/near-tier entry inside the block
  int cap;            // capacity (terms) of the workspace
  double sr, si;      // sigma = s / c
  int64_t ws;         // workspace offset in bytes
};

// status bits of one ACA
enum : int { ST_CONVERGED = 1, ST_CAPPED = 2, ST_OVERFLOW = 4, ST_EXACT = 8, ST_DEFERRED = 16 };

// workspace layout of one ACA (bytes from its start):
//   U  [cap][m] cpx<T>, W [cap][n] cpx<T>   (A ~ sum_l u_l w_l^T, V = conj(W))
//   GU [cap][cap] cpx<double>, GV [cap][cap] cpx<double>
template <typename T>
__host__ __device__ inline int64_t ws_gram_off(int cap, int m, int n) {
  int64_t a = int64_t(cap) * (m + n) * int64_t(sizeof(cpx<T>));
  return (a + 255) & ~int64_t(255);
}
template <typename T>
__host__ __device__ inline int64_t ws_bytes(int cap, int m, int n) {
  return ws_gram_off<T>(cap, m, n) + 2 * int64_t(cap) * cap * 16;
}

template <typename T>
struct AcaShared {
  unsigned used[ACA_MAXM / 32];
  cpx<T> ubuf[64];
};

struct RecompShared {
  double lam[64], sg[64];
  int keep[64], order[64];
  int nkeep, tcut;
  // one round of the parallel Jacobi ordering: pair i rotates (jp[i], jq[i])
  int jp[32], jq[32];
  double jc[32], js[32], ja[32], jd[32], jtb[32];
  cpx<double> je[32];
};

// ---- ACA of an entry function --------------------------------------------------
// Ent: prep_row(i) / prep_col(j) (group-collective, may be empty) and
// operator()(i, j) -> cpx<T>.  Partial pivoting: row residual -> pivot column
// (largest modulus, lowest index on ties) -> column residual -> Frobenius norm
// of the approximant updated with the cross terms (u_l^H u_k)(w_l^H w_k) ->
// stop when |u_k||w_k| <= tol |S_k| (term kept) -> next row = largest |u_k|
// among unused rows; a zero residual row moves on to the lowest unused row.
// Vectors in T, norms and inner products in double; the inner products are
// the Gram matrices GU = U^H U and GV = V^H V (V = conj(W)), stored for the
// recompression.  Returns the rank; `status` receives ST_* bits.
// nu: absolute norm floor of the stopping test (0: relative to the block itself)
// NW wave64s of the workgroup run the approximation together: rows and
// columns are split over all threads, each Gram entry is summed by one wave.
template <int NW, typename T, typename Ent>
__device__ int aca_grp(Ent& ent, int m, int n, int cap, int max_rank, double tol, double nu,
                       cpx<T>* __restrict__ U, cpx<T>* __restrict__ W,
                       cpx<double>* __restrict__ GU, cpx<double>* __restrict__ GV,
                       AcaShared<T>& sm, int& status) {
  constexpr int NT = NW * WAVE;
  const int tid = threadIdx.x;
  const int lane = tid & (WAVE - 1), wid = tid / WAVE;
  for (int w = tid; w < (m + 31) / 32; w += NT) sm.used[w] = 0u;
  __syncthreads();
  const int kmax = min(min(m, n), cap);
  int k = 0, i = 0, nused = 0;
  status = 0;
  double norm2 = 0.0;
  while (k < kmax) {
    // row residual of row i into W[k]
    ent.prep_row(i);
    for (int l = tid; l < k; l += NT) sm.ubuf[l] = U[int64_t(l) * m + i];
    __syncthreads();
    double best = -1.0;
    int bj = 0x7fffffff;
    for (int j = tid; j < n; j += NT) {
      cpx<T> a = ent(i, j);
      for (int l = 0; l < k; ++l) {
        cpx<T> p = cmul(sm.ubuf[l], W[int64_t(l) * n + j]);
        a.re -= p.re;
        a.im -= p.im;
      }
      W[int64_t(k) * n + j] = a;
      double v = mag2(a);
      if (v > best) { best = v; bj = j; }
    }
    if (tid == 0) sm.used[i >> 5] |= 1u << (i & 31);
    ++nused;
    grp_argmax<NW>(best, bj);
    __syncthreads();
    if (!(best > PivFloor<T>::v)) {
      int cand = 0x7fffffff;
      for (int w = tid; w < (m + 31) / 32; w += NT) {
        unsigned free_bits = ~sm.used[w];
        if (w == (m - 1) / 32 && (m & 31)) free_bits &= (1u << (m & 31)) - 1u;
        if (free_bits) cand = min(cand, w * 32 + __ffs(free_bits) - 1);
      }
      cand = grp_min_int<NW>(cand);
      if (cand == 0x7fffffff || nused >= m) { status |= ST_EXACT; break; }
      i = cand;
      continue;
    }
    const int jstar = bj;
    const cpx<T> inv = cinv(W[int64_t(k) * n + jstar]);
    __syncthreads();   // every thread has read the pivot before it is overwritten
    double nw2 = 0.0;
    for (int j = tid; j < n; j += NT) {
      cpx<T> w = (j == jstar) ? cpx<T>{T(1), T(0)} : cmul(W[int64_t(k) * n + j], inv);
      W[int64_t(k) * n + j] = w;
      nw2 += double(w.re) * double(w.re) + double(w.im) * double(w.im);
    }
    __syncthreads();
    ent.prep_col(jstar);
    for (int l = tid; l < k; l += NT) sm.ubuf[l] = W[int64_t(l) * n + jstar];
    __syncthreads();
    // column residual of column jstar into U[k]; candidate next row
    double nu2 = 0.0;
    double bestu = -1.0;
    int bi = 0x7fffffff;
    for (int r = tid; r < m; r += NT) {
      cpx<T> a = ent(r, jstar);
      for (int l = 0; l < k; ++l) {
        cpx<T> p = cmul(sm.ubuf[l], U[int64_t(l) * m + r]);
        a.re -= p.re;
        a.im -= p.im;
      }
      U[int64_t(k) * m + r] = a;
      nu2 += double(a.re) * double(a.re) + double(a.im) * double(a.im);
      if (!((sm.used[r >> 5] >> (r & 31)) & 1u)) {
        double v = mag2(a);
        if (v > bestu) { bestu = v; bi = r; }
      }
    }
    __syncthreads();
    grp_sum2<NW>(nw2, nu2);
    // Gram entries of the new term: entry l by wave l mod NW
    double crossw = 0.0;
    for (int l = wid; l < k; l += NW) {
      double gur = 0, gui = 0, gwr = 0, gwi = 0;
      for (int r = lane; r < m; r += WAVE) {
        cpx<T> a = U[int64_t(l) * m + r], b = U[int64_t(k) * m + r];
        gur += double(a.re) * b.re + double(a.im) * b.im;
        gui += double(a.re) * b.im - double(a.im) * b.re;
      }
      for (int j = lane; j < n; j += WAVE) {
        cpx<T> a = W[int64_t(l) * n + j], b = W[int64_t(k) * n + j];
        gwr += double(a.re) * b.re + double(a.im) * b.im;
        gwi += double(a.re) * b.im - double(a.im) * b.re;
      }
      gur = wave_sum(gur);
      gui = wave_sum(gui);
      gwr = wave_sum(gwr);
      gwi = wave_sum(gwi);
      crossw += gur * gwr - gui * gwi;  // Re((u_l^H u_k)(w_l^H w_k))
      if (lane == 0) {
        GU[l * cap + k] = {gur, gui};
        GU[k * cap + l] = {gur, -gui};
        // G_V[a][b] = sum_j W[a][j] conj(W[b][j]) = conj(w_a^H w_b)
        GV[l * cap + k] = {gwr, -gwi};
        GV[k * cap + l] = {gwr, gwi};
      }
    }
    const double cross = grp_sum<NW>(lane == 0 ? crossw : 0.0);
    if (tid == 0) {
      GU[k * cap + k] = {nu2, 0.0};
      GV[k * cap + k] = {nw2, 0.0};
    }
    norm2 += 2.0 * cross + nu2 * nw2;
    ++k;
    if (sqrt(nu2 * nw2) <= tol * fmax(sqrt(fmax(norm2, 0.0)), nu)) {
      status |= ST_CONVERGED;
      break;
    }
    grp_argmax<NW>(bestu, bi);
    if (nused >= m || bi == 0x7fffffff) { status |= ST_EXACT; break; }
    i = bi;
  }
  if (k == kmax && !(status & (ST_CONVERGED | ST_EXACT))) {
    if (kmax == min(m, n)) status |= ST_EXACT;
    else if (cap >= max_rank) status |= ST_CAPPED;
    else status |= ST_OVERFLOW;
  }
  __syncthreads();
  return k;
}

template <typename T, typename Ent>
__device__ inline int aca_wave(Ent& ent, int m, int n, int cap, int max_rank, double tol, double nu,
                               cpx<T>* __restrict__ U, cpx<T>* __restrict__ W,
                               cpx<double>* __restrict__ GU, cpx<double>* __restrict__ GV,
                               AcaShared<T>& sm, int& status) {
  return aca_grp<1, T, Ent>(ent, m, n, cap, max_rank, tol, nu, U, W, GU, GV, sm, status);
}

// ---- Hermitian Jacobi eigen-solver, one group, k <= 64 ------------------------
// A (k x k, row-major, generic memory) is overwritten by its eigenvalues on the
// diagonal; Q (k x k) receives the eigenvectors as columns.  Each rotation is
// G = diag(1, conj(e)) R(c, s), which zeroes A[p][q] = |b| e with the real
// rotation of the symmetric 2 x 2 problem [[a, |b|], [|b|, d]].  Sweeps use the
// round-robin (tournament) ordering: every round rotates k/2 disjoint index
// pairs at once, so a sweep is k - 1 parallel rounds instead of k (k - 1) / 2
// sequential rotations.  Rotations of one round commute (disjoint pairs), so the
// result equals the cyclic sweep in that pair order.
template <int NW>
__device__ inline void jacobi_grp(cpx<double>* A, cpx<double>* Q, int k, RecompShared& rs) {
  constexpr int NT = NW * WAVE;
  const int tid = threadIdx.x;
  for (int r = tid; r < k * k; r += NT) Q[r] = {(r / k == r % k) ? 1.0 : 0.0, 0.0};
  __syncthreads();
  if (k < 2) return;
  const int ke = (k + 1) & ~1;   // even number of positions (one dummy when k is odd)
  const int np = ke / 2;
  for (int sweep = 0; sweep < 40; ++sweep) {
    double off = 0.0, dg = 0.0;
    for (int r = tid; r < k * k; r += NT) {
      double v = cabs2(A[r]);
      if (r / k == r % k) dg += v;
      else off += v;
    }
    grp_sum2<NW>(off, dg);
    if (off <= 1e-30 * dg || off == 0.0) break;
    for (int round = 0; round < ke - 1; ++round) {
      if (tid < np) {
        // circle method: position 0 fixed, positions 1..ke-1 rotate
        auto idx = [&](int pos) { return pos == 0 ? 0 : 1 + (pos - 1 + round) % (ke - 1); };
        int p = idx(tid), q = idx(ke - 1 - tid);
        if (p > q) { int t = p; p = q; q = t; }
        double c = 1.0, sv = 0.0, a = 0.0, d = 0.0, tb = 0.0;
        cpx<double> e = {1.0, 0.0};
        if (q < k) {
          const cpx<double> b = A[p * k + q];
          a = A[p * k + p].re;
          d = A[q * k + q].re;
          const double bb = sqrt(cabs2(b));
          if (bb > 1e-300 && bb * bb > 1e-34 * fabs(a * d)) {
            const double tau = (d - a) / (2.0 * bb);
            const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
            c = 1.0 / sqrt(1.0 + t * t);
            sv = t * c;
            e = {b.re / bb, b.im / bb};
            tb = t * bb;
          } else {
            q = k;   // nothing to rotate
          }
        }
        rs.jp[tid] = p;
        rs.jq[tid] = q;
        rs.jc[tid] = c;
        rs.js[tid] = sv;
        rs.je[tid] = e;
        rs.ja[tid] = a;
        rs.jd[tid] = d;
        rs.jtb[tid] = tb;
      }
      __syncthreads();
      // columns p, q of A and Q, every row
      for (int x = tid; x < k * np; x += NT) {
        const int r = x / np, i = x % np;
        const int p = rs.jp[i], q = rs.jq[i];
        if (q >= k) continue;
        const double c = rs.jc[i], sv = rs.js[i];
        const cpx<double> ec = {rs.je[i].re, -rs.je[i].im};
        cpx<double> u = A[r * k + p], v = A[r * k + q];
        cpx<double> ev = cmul(ec, v);
        A[r * k + p] = {c * u.re - sv * ev.re, c * u.im - sv * ev.im};
        A[r * k + q] = {sv * u.re + c * ev.re, sv * u.im + c * ev.im};
        u = Q[r * k + p];
        v = Q[r * k + q];
        ev = cmul(ec, v);
        Q[r * k + p] = {c * u.re - sv * ev.re, c * u.im - sv * ev.im};
        Q[r * k + q] = {sv * u.re + c * ev.re, sv * u.im + c * ev.im};
      }
      __syncthreads();
      // rows p, q of A, every column
      for (int x = tid; x < k * np; x += NT) {
        const int r = x / np, i = x % np;
        const int p = rs.jp[i], q = rs.jq[i];
        if (q >= k) continue;
        const double c = rs.jc[i], sv = rs.js[i];
        const cpx<double> e = rs.je[i];
        cpx<double> u = A[p * k + r], v = A[q * k + r];
        cpx<double> ev = cmul(e, v);
        A[p * k + r] = {c * u.re - sv * ev.re, c * u.im - sv * ev.im};
        A[q * k + r] = {sv * u.re + c * ev.re, sv * u.im + c * ev.im};
      }
      __syncthreads();
      if (tid < np && rs.jq[tid] < k) {
        const int p = rs.jp[tid], q = rs.jq[tid];
        A[p * k + q] = {0.0, 0.0};
        A[q * k + p] = {0.0, 0.0};
        A[p * k + p] = {rs.ja[tid] - rs.jtb[tid], 0.0};
        A[q * k + q] = {rs.jd[tid] + rs.jtb[tid], 0.0};
      }
      __syncthreads();
    }
  }
  __syncthreads();
}

// ---- recompression of k ACA terms ------------------------------------------------
// GU, GV: Gram matrices (leading dimension cap).  mats: 4 k^2 doubles-complex of
// working memory (LDS or global).  Keeps the smallest t with
// sqrt(sum_{i >= t} s_i^2) <= tol max(sqrt(sum s_i^2), nu) and writes the coefficients
// CU = Q L^{1/2} Z_t and CV = Q L^{-1/2} Z_t (k x t, leading dimension t) over GU
// and GV.  Without recompression CU = CV = I, t = k.  Returns t.
template <int NW>
__device__ inline int recompress_grp(int k, int cap, cpx<double>* GU, cpx<double>* GV, double tol,
                                     double nu, bool do_recompress, cpx<double>* mats,
                                     RecompShared& rs) {
  constexpr int NT = NW * WAVE;
  const int tid = threadIdx.x;
  if (k == 0 || !do_recompress) {
    __syncthreads();
    for (int r = tid; r < k * k; r += NT) {
      GU[r] = {(r / k == r % k) ? 1.0 : 0.0, 0.0};
      GV[r] = GU[r];
    }
    __syncthreads();
    return k;
  }
  cpx<double>* A = mats;
  cpx<double>* Q = A + k * k;
  cpx<double>* B = Q + k * k;
  cpx<double>* Z = B + k * k;
  for (int r = tid; r < k * k; r += NT) A[r] = GV[(r / k) * cap + (r % k)];
  __syncthreads();
  jacobi_grp<NW>(A, Q, k, rs);
  if (tid < k) rs.lam[tid] = A[tid * k + tid].re;
  __syncthreads();
  double lmax = 0.0;
  for (int a = 0; a < k; ++a) lmax = fmax(lmax, rs.lam[a]);
  if (tid == 0) {
    int c = 0;
    for (int a = 0; a < k; ++a)
      if (rs.lam[a] > 1e-14 * lmax && rs.lam[a] > 0.0) rs.keep[c++] = a;
    rs.nkeep = c;
  }
  __syncthreads();
  const int kk = rs.nkeep;
  if (kk == 0) return 0;
  // T1 = GU Q_S (k x kk) into Z, then B = L^1/2 Q_S^H T1 L^1/2
  for (int e = tid; e < k * kk; e += NT) {
    const int x = e / kk, b = e % kk;
    const int qb = rs.keep[b];
    cpx<double> acc = {0, 0};
    for (int y = 0; y < k; ++y) {
      cpx<double> p = cmul(GU[x * cap + y], Q[y * k + qb]);
      acc.re += p.re;
      acc.im += p.im;
    }
    Z[x * kk + b] = acc;
  }
  __syncthreads();
  for (int e = tid; e < kk * kk; e += NT) {
    const int a = e / kk, b = e % kk;
    const int qa = rs.keep[a];
    cpx<double> acc = {0, 0};
    for (int x = 0; x < k; ++x) {
      cpx<double> p = cmulc(Q[x * k + qa], Z[x * kk + b]);
      acc.re += p.re;
      acc.im += p.im;
    }
    const double sc = sqrt(rs.lam[qa] * rs.lam[rs.keep[b]]);
    B[a * kk + b] = {acc.re * sc, acc.im * sc};
  }
  __syncthreads();
  for (int e = tid; e < kk * kk; e += NT) {  // Hermitian part
    const int a = e / kk, b = e % kk;
    if (a < b) {
      cpx<double> x = B[a * kk + b], y = B[b * kk + a];
      cpx<double> h = {0.5 * (x.re + y.re), 0.5 * (x.im - y.im)};
      B[a * kk + b] = h;
      B[b * kk + a] = {h.re, -h.im};
    } else if (a == b) {
      B[a * kk + a].im = 0.0;
    }
  }
  __syncthreads();
  jacobi_grp<NW>(B, Z, kk, rs);
  if (tid < kk) rs.sg[tid] = fmax(B[tid * kk + tid].re, 0.0);
  __syncthreads();
  if (tid < kk) {  // descending order, ties by index
    int pos = 0;
    for (int b = 0; b < kk; ++b)
      if (rs.sg[b] > rs.sg[tid] || (rs.sg[b] == rs.sg[tid] && b < tid)) ++pos;
    rs.order[pos] = tid;
  }
  __syncthreads();
  if (tid == 0) {
    double total = 0.0;
    for (int a = 0; a < kk; ++a) total += rs.sg[a];
    double tail = 0.0;
    int t = kk;
    const double ref = fmax(sqrt(total), nu);
    for (int a = kk - 1; a >= 0; --a) {
      tail += rs.sg[rs.order[a]];
      if (sqrt(tail) <= tol * ref) t = a;
      else break;
    }
    rs.tcut = t;
  }
  __syncthreads();
  const int t = rs.tcut;
  for (int e = tid; e < k * t; e += NT) {
    const int x = e / t, c = e % t;
    const int zc = rs.order[c];
    cpx<double> au = {0, 0}, av = {0, 0};
    for (int a = 0; a < kk; ++a) {
      const int qa = rs.keep[a];
      cpx<double> p = cmul(Q[x * k + qa], Z[a * kk + zc]);
      const double sl = sqrt(rs.lam[qa]);
      au.re += p.re * sl;
      au.im += p.im * sl;
      av.re += p.re / sl;
      av.im += p.im / sl;
    }
    A[e] = au;  // A and B are free now
    B[e] = av;
  }
  __syncthreads();
  for (int e = tid; e < k * t; e += NT) {
    GU[e] = A[e];
    GV[e] = B[e];
  }
  __syncthreads();
  return t;
}

__device__ inline int recompress_wave(int k, int cap, cpx<double>* GU, cpx<double>* GV, double tol,
                                      double nu, bool do_recompress, cpx<double>* mats,
                                      RecompShared& rs) {
  return recompress_grp<1>(k, cap, GU, GV, tol, nu, do_recompress, mats, rs);
}

// ---- Ubar = U CU (m x t), Vbar = conj(W) CV (n x t), column-major outputs ----------
template <typename T>
__device__ inline void apply_factors(int k, int t, int m, int n, const cpx<T>* U, const cpx<T>* W,
                                     const cpx<double>* CU, const cpx<double>* CV, cpx<T>* OU,
                                     cpx<T>* OV, int tid, int nthreads) {
  const int64_t total = int64_t(m + n) * t;
  for (int64_t e = tid; e < total; e += nthreads) {
    if (e < int64_t(m) * t) {
      const int c = int(e / m), r = int(e % m);
      cpx<double> acc = {0, 0};
      for (int x = 0; x < k; ++x) {
        cpx<T> u = U[int64_t(x) * m + r];
        cpx<double> cu = CU[x * t + c];
        acc.re += double(u.re) * cu.re - double(u.im) * cu.im;
        acc.im += double(u.re) * cu.im + double(u.im) * cu.re;
      }
      OU[int64_t(c) * m + r] = {T(acc.re), T(acc.im)};
    } else {
      const int64_t e2 = e - int64_t(m) * t;
      const int c = int(e2 / n), j = int(e2 % n);
      cpx<double> acc = {0, 0};
      for (int x = 0; x < k; ++x) {
        cpx<T> w = W[int64_t(x) * n + j];  // V[j][x] = conj(w)
        cpx<double> cv = CV[x * t + c];
        acc.re += double(w.re) * cv.re + double(w.im) * cv.im;
        acc.im += double(w.re) * cv.im - double(w.im) * cv.re;
      }
      OV[int64_t(c) * n + j] = {T(acc.re), T(acc.im)};
    }
  }
}

}  // namespace gcq
