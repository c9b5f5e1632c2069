// Wave-level routines for the low-rank face of Sec. 4, shared by the per-
// frequency ACA kernels and the 3D-ACA kernel.
//
// aca_wave: partially pivoted ACA of an entry function (one wave64).
// recompress_wave: QR/SVD recompression of the ACA factors, carried out
//   through their Gram matrices: G_V = V^H V = R^H R by Cholesky with
//   diagonal pivoting (R, upper triangular on its pivot order, plays the role
//   of the QR factor of V; a remaining diagonal below 1e-14 of the largest
//   ends it at numerical rank r), then B = R G_U R^H = Z S^2 Z^H by Hermitian
//   Jacobi, so that S holds the singular values of U V^H; the truncated
//   factors are Ubar = U R^H Z_t and Vbar = V R^+ Z_t, R^+ the right inverse
//   of R on its pivot rows (a triangular solve).
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
  int nrows;   // rows evaluated by the last approximation
};

// shared state of one recompression of at most MK terms
template <int MK>
struct RecompSharedT {
  static constexpr int NP = (MK + 1) / 2;   // index pairs of a Jacobi round
  double sg[MK];
  int keep[MK], order[MK];
  int nkeep, tcut;
  // one round of the parallel Jacobi ordering, per index pair i: the rotation
  // {c, s, Re e, Im e} (the identity when the pair is not rotated), the new
  // diagonal of the pair's 2 x 2 block, and the pair's indices p | q << 8
  double4 rot[NP];
  double2 dia[NP];
  int pq[NP];
  double dmax;
};
using RecompShared = RecompSharedT<64>;

// working memory of the recompression of k terms (complex doubles)
__host__ __device__ constexpr int recompress_mats(int k) { return 3 * k * k; }

// The reductions that end an ACA step, in one exchange: group sums of a and b
// (per-thread partials), of c (a value each wave already holds summed), and
// the group argmax of (val, idx) (largest val, lowest idx on ties).  Waves
// are combined in wave order, so the results do not depend on timing.  The
// exchange slots are this function's own; the barriers between two calls of
// one ACA step keep their readers apart.
template <int NW>
__device__ __forceinline__ void grp_step_reduce(double& a, double& b, double& c, double& val,
                                                int& idx) {
  a = wave_sum(a);
  b = wave_sum(b);
  wave_argmax(val, idx);
  if constexpr (NW > 1) {
    __shared__ double ra[NW], rb[NW], rc[NW], rv[NW];
    __shared__ int ri[NW];
    if ((threadIdx.x & (WAVE - 1)) == 0) {
      const int w = threadIdx.x / WAVE;
      ra[w] = a;
      rb[w] = b;
      rc[w] = c;
      rv[w] = val;
      ri[w] = idx;
    }
    __syncthreads();
    a = ra[0];
    b = rb[0];
    c = rc[0];
    val = rv[0];
    idx = ri[0];
#pragma unroll
    for (int w = 1; w < NW; ++w) {
      a += ra[w];
      b += rb[w];
      c += rc[w];
      if (rv[w] > val || (rv[w] == val && ri[w] < idx)) {
        val = rv[w];
        idx = ri[w];
      }
    }
  }
}

// ---- ACA of an entry function --------------------------------------------------
// Ent: prep_row(i) / prep_col(j) (group-collective, may be empty) and
// part(i, j, p, P) -> cpx<T>, part p of P of the entry (i, j), the parts of
// the P lanes adding up to the entry.  Partial pivoting: row residual -> pivot column
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
// SPLIT: rows shorter than the group spread each entry over several lanes.
template <int NW, bool SPLIT, typename T, typename Ent>
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
    if constexpr (!SPLIT) {
      for (int j = tid; j < n; j += NT) {
        cpx<T> a = ent.part(i, j, 0, 1);
        for (int l = 0; l < k; ++l) {
          cpx<T> q = cmul(sm.ubuf[l], W[int64_t(l) * n + j]);
          a.re -= q.re;
          a.im -= q.im;
        }
        W[int64_t(k) * n + j] = a;
        double v = mag2(a);
        if (v > best) { best = v; bj = j; }
      }
    } else {
      // P lanes per entry when the row is short: they split the quadrature
      // points and the residual sums
      const int P = split_lanes(NT, n), E = NT / P, p = tid % P;
      for (int j0 = 0; j0 < n; j0 += E) {
        const int j = j0 + tid / P;
        const bool ok = j < n;
        cpx<T> a = {T(0), T(0)};
        if (ok) {
          a = ent.part(i, j, p, P);
          for (int l = p; l < k; l += P) {
            cpx<T> q = cmul(sm.ubuf[l], W[int64_t(l) * n + j]);
            a.re -= q.re;
            a.im -= q.im;
          }
        }
        a = lanes_sum(a, P);
        if (ok && p == 0) {
          W[int64_t(k) * n + j] = a;
          double v = mag2(a);
          if (v > best) { best = v; bj = j; }
        }
      }
    }
    if (tid == 0) sm.used[i >> 5] |= 1u << (i & 31);
    ++nused;
    grp_argmax<NW>(best, bj);
    best = unid(best);
    bj = uni(bj);
    __syncthreads();
    if (!(best > PivFloor<T>::v)) {
      int cand = 0x7fffffff;
      for (int w = tid; w < (m + 31) / 32; w += NT) {
        unsigned free_bits = ~sm.used[w];
        if (w == (m - 1) / 32 && (m & 31)) free_bits &= (1u << (m & 31)) - 1u;
        if (free_bits) cand = min(cand, w * 32 + __ffs(free_bits) - 1);
      }
      cand = uni(grp_min_int<NW>(cand));
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
    if constexpr (!SPLIT) {
      for (int r = tid; r < m; r += NT) {
        cpx<T> a = ent.part(r, jstar, 0, 1);
        for (int l = 0; l < k; ++l) {
          cpx<T> q = cmul(sm.ubuf[l], U[int64_t(l) * m + r]);
          a.re -= q.re;
          a.im -= q.im;
        }
        U[int64_t(k) * m + r] = a;
        nu2 += double(a.re) * double(a.re) + double(a.im) * double(a.im);
        if (!((sm.used[r >> 5] >> (r & 31)) & 1u)) {
          double v = mag2(a);
          if (v > bestu) { bestu = v; bi = r; }
        }
      }
    } else {
      const int P = split_lanes(NT, m), E = NT / P, p = tid % P;
      for (int r0 = 0; r0 < m; r0 += E) {
        const int r = r0 + tid / P;
        const bool ok = r < m;
        cpx<T> a = {T(0), T(0)};
        if (ok) {
          a = ent.part(r, jstar, p, P);
          for (int l = p; l < k; l += P) {
            cpx<T> q = cmul(sm.ubuf[l], U[int64_t(l) * m + r]);
            a.re -= q.re;
            a.im -= q.im;
          }
        }
        a = lanes_sum(a, P);
        if (ok && p == 0) {
          U[int64_t(k) * m + r] = a;
          nu2 += double(a.re) * double(a.re) + double(a.im) * double(a.im);
          if (!((sm.used[r >> 5] >> (r & 31)) & 1u)) {
            double v = mag2(a);
            if (v > bestu) { bestu = v; bi = r; }
          }
        }
      }
    }
    __syncthreads();
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
    // one exchange for |w_k|^2, |u_k|^2, the cross terms and the next row
    grp_step_reduce<NW>(nw2, nu2, crossw, bestu, bi);
    nw2 = unid(nw2);
    nu2 = unid(nu2);
    const double cross = unid(crossw);
    bi = uni(bi);
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
    if (nused >= m || bi == 0x7fffffff) { status |= ST_EXACT; break; }
    i = bi;
  }
  if (k == kmax && !(status & (ST_CONVERGED | ST_EXACT))) {
    if (kmax == min(m, n)) status |= ST_EXACT;
    else if (cap >= max_rank) status |= ST_CAPPED;
    else status |= ST_OVERFLOW;
  }
  if (tid == 0) sm.nrows = nused;
  __syncthreads();
  return k;
}

template <typename T, typename Ent>
__device__ inline int aca_wave(Ent& ent, int m, int n, int cap, int max_rank, double tol, double nu,
                               cpx<T>* __restrict__ U, cpx<T>* __restrict__ W,
                               cpx<double>* __restrict__ GU, cpx<double>* __restrict__ GV,
                               AcaShared<T>& sm, int& status) {
  return aca_grp<1, false, T, Ent>(ent, m, n, cap, max_rank, tol, nu, U, W, GU, GV, sm, status);
}

// ---- Hermitian Jacobi eigen-solver, one group, k <= 64 ------------------------
// A (k x k, row-major, generic memory) is overwritten by its eigenvalues on the
// diagonal; Q (k x k) receives the eigenvectors as columns.  Each rotation is
// G = diag(1, conj(e)) R(c, s), which zeroes A[p][q] = |b| e with the real
// rotation of the symmetric 2 x 2 problem [[a, |b|], [|b|, d]].  Sweeps use the
// round-robin (tournament) ordering: every round rotates k/2 disjoint index
// pairs at once, so a sweep is k - 1 parallel rounds instead of k (k - 1) / 2
// sequential rotations.  Rotations of one round commute (disjoint pairs), so the
// result equals the cyclic sweep in that pair order.  A round is three phases:
// the rotation parameters (a pair whose |b|^2 is below 1e-34 |a d| is not
// rotated: its b is set to zero, a change below the rounding of a and d), then
// G^H A G by 2 x 2 blocks (rows of pair i, columns of pair j) and Q G by rows,
// each thread applying the rotations of its blocks without branches (the
// identity for pairs not rotated).  Sweeps stop when the off-diagonal squared
// Frobenius norm is at most `thr` times the diagonal's.
// Always inlined: callers pass A and Q either in LDS or in global memory, and
// the accesses compile to LDS instructions only where the pointer's origin is
// visible.
template <int NW, typename RS>
__device__ __attribute__((always_inline)) inline void jacobi_grp(cpx<double>* A, cpx<double>* Q,
                                                                 int k, RS& rs, double thr) {
  constexpr int NT = NW * WAVE;
  const int tid = threadIdx.x;
  for (int r = tid; r < k * k; r += NT) Q[r] = {(r / k == r % k) ? 1.0 : 0.0, 0.0};
  __syncthreads();
  if (k < 2) return;
  const int ke = (k + 1) & ~1;   // even number of positions (one dummy when k is odd)
  const int np = ke / 2;
  // work items of the update phases: (i, j) = (x / np, x % np) for x = tid,
  // tid + NT, ...; decomposed once and advanced with a carry
  const int row0 = tid / np, j0 = tid % np, drow = NT / np, dj = NT % np;
  for (int sweep = 0; sweep < 40; ++sweep) {
    double off = 0.0, dg = 0.0;
    for (int r = tid; r < k * k; r += NT) {
      double v = cabs2(A[r]);
      if (r / k == r % k) dg += v;
      else off += v;
    }
    grp_sum2<NW>(off, dg);
    if (off <= thr * dg || off == 0.0) break;
    for (int round = 0; round < ke - 1; ++round) {
      if (tid < np) {
        // circle method: position 0 fixed, positions 1..ke-1 rotate
        auto idx = [&](int pos) {
          if (pos == 0) return 0;
          int v = pos - 1 + round;   // < 2 (ke - 1)
          if (v >= ke - 1) v -= ke - 1;
          return 1 + v;
        };
        int p = idx(tid), q = idx(ke - 1 - tid);
        if (p > q) { int t = p; p = q; q = t; }
        double c = 1.0, sv = 0.0, a = 0.0, d = 0.0, tb = 0.0;
        cpx<double> e = {1.0, 0.0};
        if (q < k) {
          const cpx<double> b = A[p * k + q];
          a = A[p * k + p].re;
          d = A[q * k + q].re;
          const double bb2 = cabs2(b);
          if (bb2 > 1e-300 && bb2 > 1e-34 * fabs(a * d)) {
            const double ib = rsqrt(bb2);   // 1 / |b|
            const double tau = 0.5 * (d - a) * ib;
            const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
            c = rsqrt(1.0 + t * t);
            sv = t * c;
            e = {b.re * ib, b.im * ib};
            tb = t * (bb2 * ib);
          }
        }
        rs.rot[tid] = {c, sv, e.re, e.im};
        rs.dia[tid] = {a - tb, d + tb};
        rs.pq[tid] = p | (q << 8);
      }
      __syncthreads();
      {   // G^H A G: block (rows of pair i, columns of pair j)
        int i = row0, j = j0;
        for (int x = tid; x < np * np; x += NT) {
          const int ci = i, cj = j;
          i += drow;
          j += dj;
          if (j >= np) { j -= np; ++i; }
          const int pqi = rs.pq[ci], pqj = rs.pq[cj];
          const int pi = pqi & 255, qi = pqi >> 8, pj = pqj & 255, qj = pqj >> 8;
          const bool qiv = qi < k, qjv = qj < k;
          if (ci == cj) {   // the pair's own block becomes diagonal
            if (qiv) {
              const double2 dd = rs.dia[ci];
              A[pi * k + qi] = {0.0, 0.0};
              A[qi * k + pi] = {0.0, 0.0};
              A[pi * k + pi] = {dd.x, 0.0};
              A[qi * k + qi] = {dd.y, 0.0};
            }
            continue;
          }
          cpx<double> app = A[pi * k + pj];
          cpx<double> apq = qjv ? A[pi * k + qj] : cpx<double>{0.0, 0.0};
          cpx<double> aqp = qiv ? A[qi * k + pj] : cpx<double>{0.0, 0.0};
          cpx<double> aqq = qiv && qjv ? A[qi * k + qj] : cpx<double>{0.0, 0.0};
          {   // columns: [u, v] -> [c u - s conj(e) v, s u + c conj(e) v]
            const double4 R = rs.rot[cj];
            const cpx<double> ec = {R.z, -R.w};
            cpx<double> ev = cmul(ec, apq);
            const cpx<double> n0 = {R.x * app.re - R.y * ev.re, R.x * app.im - R.y * ev.im};
            const cpx<double> n1 = {R.y * app.re + R.x * ev.re, R.y * app.im + R.x * ev.im};
            ev = cmul(ec, aqq);
            const cpx<double> n2 = {R.x * aqp.re - R.y * ev.re, R.x * aqp.im - R.y * ev.im};
            const cpx<double> n3 = {R.y * aqp.re + R.x * ev.re, R.y * aqp.im + R.x * ev.im};
            app = n0; apq = n1; aqp = n2; aqq = n3;
          }
          {   // rows: [u; v] -> [c u - s e v; s u + c e v]
            const double4 R = rs.rot[ci];
            const cpx<double> e = {R.z, R.w};
            cpx<double> ev = cmul(e, aqp);
            const cpx<double> n0 = {R.x * app.re - R.y * ev.re, R.x * app.im - R.y * ev.im};
            const cpx<double> n2 = {R.y * app.re + R.x * ev.re, R.y * app.im + R.x * ev.im};
            ev = cmul(e, aqq);
            const cpx<double> n1 = {R.x * apq.re - R.y * ev.re, R.x * apq.im - R.y * ev.im};
            const cpx<double> n3 = {R.y * apq.re + R.x * ev.re, R.y * apq.im + R.x * ev.im};
            app = n0; apq = n1; aqp = n2; aqq = n3;
          }
          A[pi * k + pj] = app;
          if (qjv) A[pi * k + qj] = apq;
          if (qiv) A[qi * k + pj] = aqp;
          if (qiv && qjv) A[qi * k + qj] = aqq;
        }
      }
      {   // Q G: row r, columns of pair j
        int r = row0, j = j0;
        for (int x = tid; x < k * np; x += NT) {
          const int cr = r, cj = j;
          r += drow;
          j += dj;
          if (j >= np) { j -= np; ++r; }
          const int pqj = rs.pq[cj];
          const int p = pqj & 255, q = pqj >> 8;
          if (q >= k) continue;
          const double4 R = rs.rot[cj];
          const cpx<double> ec = {R.z, -R.w};
          const cpx<double> u = Q[cr * k + p], v = Q[cr * k + q];
          const cpx<double> ev = cmul(ec, v);
          Q[cr * k + p] = {R.x * u.re - R.y * ev.re, R.x * u.im - R.y * ev.im};
          Q[cr * k + q] = {R.y * u.re + R.x * ev.re, R.y * u.im + R.x * ev.im};
        }
      }
      __syncthreads();
    }
  }
  __syncthreads();
}

// ---- recompression of k ACA terms ------------------------------------------------
// GU, GV: Gram matrices (leading dimension cap).  mats: recompress_mats(k)
// complex doubles of working memory (LDS or global).
//   1. G_V = R^H R by Cholesky with diagonal pivoting (rows of R in pivot
//      order; a remaining diagonal below 1e-14 of the largest ends it at rank
//      r): R plays the role of the triangular factor of V = Q_V R.
//   2. B = R G_U R^H = Z S^2 Z^H (Jacobi), the core M = R_U R^H having B = M^H M.
//   3. Keep the smallest t with sqrt(sum_{i >= t} s_i^2) <= tol max(sqrt(sum s_i^2), nu):
//      Ubar = U CU, CU = R^H Z_t;  Vbar = V CV, CV = R^+ Z_t, R^+ the right
//      inverse of R supported on the pivot rows (triangular solve).
// CU and CV (k x t, leading dimension t) are written over GU and GV.  Without
// recompression CU = CV = I, t = k.  Returns t.
// Always inlined, for the reason given at jacobi_grp.
template <int NW, typename RS>
__device__ __attribute__((always_inline)) inline int recompress_grp(
    int k, int cap, cpx<double>* GU, cpx<double>* GV, double tol, double nu, bool do_recompress,
    cpx<double>* mats, RS& rs) {
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
  cpx<double>* S = mats;           // k x k Schur complement of G_V, then R (rows in pivot order)
  cpx<double>* B = S + k * k;      // r x r
  cpx<double>* Z = B + k * k;      // r x r
  cpx<double>* R = Z;              // rows of R are built in Z first (B, Z are free until step 2)
  for (int e = tid; e < k * k; e += NT) {
    S[e] = GV[(e / k) * cap + (e % k)];
    R[e] = {0.0, 0.0};
  }
  if (tid < k) rs.keep[tid] = 0;   // eliminated flags
  __syncthreads();
  if (tid < WAVE) {   // largest diagonal, by wave 0
    double d0 = 0.0;
    for (int a = tid; a < k; a += WAVE) d0 = fmax(d0, S[a * k + a].re);
    int dummy = 0;
    wave_argmax(d0, dummy);
    if (tid == 0) rs.dmax = d0;
  }
  __syncthreads();
  const double dlim = 1e-14 * unid(rs.dmax);
  int r = 0;
  for (; r < k; ++r) {
    // pivot: largest remaining diagonal (lowest index on ties), by wave 0
    if (tid < WAVE) {
      double best = -1.0;
      int p = 0x7fffffff;
      for (int a = tid; a < k; a += WAVE) {
        if (rs.keep[a]) continue;
        const double v = S[a * k + a].re;
        if (v > best) { best = v; p = a; }
      }
      wave_argmax(best, p);
      if (tid == 0) {
        if (p != 0x7fffffff && best > dlim && best > 0.0) {
          rs.nkeep = p;
          rs.keep[p] = 1;
          rs.order[r] = p;   // pivot of row r
        } else {
          rs.nkeep = -1;
        }
      }
    }
    __syncthreads();
    const int p = uni(rs.nkeep);
    if (p < 0) break;
    const double piv = sqrt(S[p * k + p].re);
    // R[r][b] = S[p][b] / piv over remaining b (R[r][p] = piv)
    for (int b2 = tid; b2 < k; b2 += NT) {
      if (rs.keep[b2] && b2 != p) continue;
      const cpx<double> v = S[p * k + b2];
      R[r * k + b2] = b2 == p ? cpx<double>{piv, 0.0} : cpx<double>{v.re / piv, v.im / piv};
    }
    __syncthreads();
    // S[a][b] -= conj(R[r][a]) R[r][b] over remaining a, b
    for (int e = tid; e < k * k; e += NT) {
      const int a = e / k, b2 = e % k;
      if (rs.keep[a] || rs.keep[b2]) continue;
      const cpx<double> x = R[r * k + a], y = R[r * k + b2];
      S[e].re -= x.re * y.re + x.im * y.im;
      S[e].im -= x.re * y.im - x.im * y.re;
    }
    __syncthreads();
  }
  if (r == 0) return 0;
  // keep R (r x k) in S, then B = R G_U R^H: T1 = G_U R^H (k x r) into Z first
  for (int e = tid; e < r * k; e += NT) S[e] = R[e];
  __syncthreads();
  for (int e = tid; e < k * r; e += NT) {
    const int x = e / r, b2 = e % r;
    cpx<double> acc = {0, 0};
    for (int y = 0; y < k; ++y) {
      const cpx<double> g = GU[x * cap + y], rr = S[b2 * k + y];
      acc.re += g.re * rr.re + g.im * rr.im;   // g conj(rr)
      acc.im += g.im * rr.re - g.re * rr.im;
    }
    Z[e] = acc;
  }
  __syncthreads();
  for (int e = tid; e < r * r; e += NT) {
    const int a = e / r, b2 = e % r;
    cpx<double> acc = {0, 0};
    for (int x = 0; x < k; ++x) {
      const cpx<double> p = cmul(S[a * k + x], Z[x * r + b2]);
      acc.re += p.re;
      acc.im += p.im;
    }
    B[e] = acc;
  }
  __syncthreads();
  for (int e = tid; e < r * r; e += NT) {  // Hermitian part
    const int a = e / r, b2 = e % r;
    if (a < b2) {
      cpx<double> x = B[a * r + b2], y = B[b2 * r + a];
      cpx<double> h = {0.5 * (x.re + y.re), 0.5 * (x.im - y.im)};
      B[a * r + b2] = h;
      B[b2 * r + a] = {h.re, -h.im};
    } else if (a == b2) {
      B[a * r + a].im = 0.0;
    }
  }
  __syncthreads();
  // B's eigenvalues s_i^2 decide the truncation at relative tol: a relative
  // off-diagonal norm of tol^2 leaves them, and the kept directions, accurate
  // to far below that (full float64, 1e-15, for tol <= 3e-8)
  const double rel_off = fmax(tol * tol, 1e-15);
  jacobi_grp<NW>(B, Z, r, rs, rel_off * rel_off);
  if (tid < r) rs.sg[tid] = fmax(B[tid * r + tid].re, 0.0);
  __syncthreads();
  if (tid < r) {  // descending order, ties by index
    int pos = 0;
    for (int b2 = 0; b2 < r; ++b2)
      if (rs.sg[b2] > rs.sg[tid] || (rs.sg[b2] == rs.sg[tid] && b2 < tid)) ++pos;
    rs.keep[pos] = tid;   // (the elimination flags are no longer needed)
  }
  __syncthreads();
  if (tid == 0) {
    double total = 0.0;
    for (int a = 0; a < r; ++a) total += rs.sg[a];
    double tail = 0.0;
    int t = r;
    const double ref = fmax(sqrt(total), nu);
    for (int a = r - 1; a >= 0; --a) {
      tail += rs.sg[rs.keep[a]];
      if (sqrt(tail) <= tol * ref) t = a;
      else break;
    }
    rs.tcut = t;
  }
  __syncthreads();
  const int t = uni(rs.tcut);
  // CU = R^H Z_t (k x t) over GU
  for (int e = tid; e < k * t; e += NT) {
    const int x = e / t, c = e % t;
    const int zc = rs.keep[c];
    cpx<double> acc = {0, 0};
    for (int a = 0; a < r; ++a) {
      const cpx<double> p = cmulc(S[a * k + x], Z[a * r + zc]);   // conj(R[a][x]) Z[a][zc]
      acc.re += p.re;
      acc.im += p.im;
    }
    GU[e] = acc;
  }
  // CV: rows order[j] of R_P^{-1} Z_t, R_P[i][j] = R[i][order[j]] upper triangular
  for (int e = tid; e < k * t; e += NT) GV[e] = {0.0, 0.0};
  __syncthreads();
  for (int c = tid; c < t; c += NT) {
    const int zc = rs.keep[c];
    for (int i = r - 1; i >= 0; --i) {
      cpx<double> acc = Z[i * r + zc];
      for (int j = i + 1; j < r; ++j) {
        const cpx<double> p = cmul(S[i * k + rs.order[j]], GV[rs.order[j] * t + c]);
        acc.re -= p.re;
        acc.im -= p.im;
      }
      const double dii = S[i * k + rs.order[i]].re;   // real positive pivot
      GV[rs.order[i] * t + c] = {acc.re / dii, acc.im / dii};
    }
  }
  __syncthreads();
  return t;
}

template <typename RS>
__device__ __attribute__((always_inline)) inline int recompress_wave(int k, int cap, cpx<double>* GU,
                                                                     cpx<double>* GV, double tol, double nu,
                                                                     bool do_recompress, cpx<double>* mats,
                                                                     RS& rs) {
  return recompress_grp<1>(k, cap, GU, GV, tol, nu, do_recompress, mats, rs);
}

// ---- Ubar = U CU (m x t), Vbar = conj(W) CV (n x t), column-major outputs ----------
// A thread owns one row of U (or W) and APPLY_COLS output columns: it reads the
// row once per APPLY_COLS columns (the coefficients are the same for all lanes
// of a wave, so they come as broadcasts); each output sums over x in the same
// order as a per-element loop would.
constexpr int APPLY_COLS = 8;
template <typename T>
__device__ __attribute__((always_inline)) inline void apply_factors(int k, int t, int m, int n, const cpx<T>* U, const cpx<T>* W,
                                     const cpx<double>* CU, const cpx<double>* CV, cpx<T>* OU,
                                     cpx<T>* OV, int tid, int nthreads) {
  const int rows = m + n;
  const int nch = (t + APPLY_COLS - 1) / APPLY_COLS;
  const int64_t total = int64_t(rows) * nch;
  for (int64_t e = tid; e < total; e += nthreads) {
    const int r = int(e % rows), c0 = int(e / rows) * APPLY_COLS;
    const int nc = min(APPLY_COLS, t - c0);
    double are[APPLY_COLS], aim[APPLY_COLS];
#pragma unroll
    for (int q = 0; q < APPLY_COLS; ++q) are[q] = aim[q] = 0.0;
    if (r < m) {
      for (int x = 0; x < k; ++x) {
        const cpx<T> u = U[int64_t(x) * m + r];
        const double ur = double(u.re), ui = double(u.im);
#pragma unroll
        for (int q = 0; q < APPLY_COLS; ++q) {
          if (q >= nc) break;
          const cpx<double> cu = CU[x * t + c0 + q];
          are[q] += ur * cu.re - ui * cu.im;
          aim[q] += ur * cu.im + ui * cu.re;
        }
      }
#pragma unroll
      for (int q = 0; q < APPLY_COLS; ++q) {
        if (q >= nc) break;
        OU[int64_t(c0 + q) * m + r] = {T(are[q]), T(aim[q])};
      }
    } else {
      const int j = r - m;
      for (int x = 0; x < k; ++x) {
        const cpx<T> w = W[int64_t(x) * n + j];   // V[j][x] = conj(w)
        const double wr = double(w.re), wi = double(w.im);
#pragma unroll
        for (int q = 0; q < APPLY_COLS; ++q) {
          if (q >= nc) break;
          const cpx<double> cv = CV[x * t + c0 + q];
          are[q] += wr * cv.re + wi * cv.im;
          aim[q] += wr * cv.im - wi * cv.re;
        }
      }
#pragma unroll
      for (int q = 0; q < APPLY_COLS; ++q) {
        if (q >= nc) break;
        OV[int64_t(c0 + q) * n + j] = {T(are[q]), T(aim[q])};
      }
    }
  }
}

}  // namespace gcq
