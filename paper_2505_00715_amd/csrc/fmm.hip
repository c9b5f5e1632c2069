// FMM-based 3D-ACA (Sec. 4, the face approximated by a black-box FMM,
// eq. cheb; Alg. 1 and eq. norm along the frequency axis).
//
// The far field of an admissible block (X, Y) is the Chebyshev interpolation
// of the kernel in both clusters' boxes:
//   A_XY(s) ~ L_X K_XY(s) R_Y^T,  L_X[i, n] = S_X(x_i, x_n),
//   R_Y[j, m] = sum_q w_jq S_Y(y_jq, y_m),  K_XY(s)[n, m] = exp(-s r / c) / (4 pi r)
// with p Chebyshev nodes (the zeros of T_p) per dimension in each cluster's
// vertex box.  Only the M2L operators K_XY(s) depend on the frequency; each
// admissible block's tensor [K_XY(s_k)]_k is compressed by Alg. 1 with dense
// slices, the same kernel the inadmissible blocks use.  The product runs the
// multi-level scheme P2M (R^T at the leaves), M2M, M2L (sum_d f_d[k] H_d),
// L2L, L2P (L at the leaves): a parent's Lagrange polynomials (degree p - 1)
// are interpolated exactly by a son's nodes, so R_P = [R_son T_son] with
// T_son[m, m'] = S_P(y_m^son, y_m'^P), and the multi-level product equals the
// single-level form up to rounding.
#include <algorithm>
#include <cmath>
#include <numeric>
#include <vector>

#include "internal.h"
#include "lowrank.h"
#include "matvec.h"

namespace gcq {

constexpr int FMM_PMAX = 6;       // nodes per dimension
constexpr int FMM_RC = 8;         // rows of the M2L output a workgroup owns
constexpr double FMM_MIN_HALF = 1e-3;

// ---- host: interpolation tables --------------------------------------------------------

static void cheb_nodes(int p, double* t) {
  for (int a = 0; a < p; ++a) t[a] = std::cos((2 * a + 1) * M_PI / (2 * p));
}

// the p Lagrange polynomials of the Chebyshev nodes at u
static void lagrange_1d(int p, const double* t, double u, double* out) {
  for (int a = 0; a < p; ++a) {
    double v = 1.0;
    for (int b = 0; b < p; ++b)
      if (b != a) v *= (u - t[b]) / (t[a] - t[b]);
    out[a] = v;
  }
}

struct FmmBox {
  double c[3], h[3];
};

static FmmBox box_of(const Cluster& C) {
  FmmBox b;
  double hmax = 0.0;
  for (int d = 0; d < 3; ++d) {
    b.c[d] = 0.5 * (C.bmin[d] + C.bmax[d]);
    b.h[d] = 0.5 * (C.bmax[d] - C.bmin[d]);
    hmax = std::max(hmax, b.h[d]);
  }
  for (int d = 0; d < 3; ++d) b.h[d] = std::max(b.h[d], FMM_MIN_HALF * hmax);
  return b;
}

// S_box(x, node n) for all p^3 nodes, n = a_x + p a_y + p^2 a_z
static void interp_row(const FmmBox& b, int p, const double* t, const double x[3], double* out) {
  double l[3][FMM_PMAX];
  for (int d = 0; d < 3; ++d) lagrange_1d(p, t, (x[d] - b.c[d]) / b.h[d], l[d]);
  for (int az = 0; az < p; ++az)
    for (int ay = 0; ay < p; ++ay)
      for (int ax = 0; ax < p; ++ax) out[ax + p * (ay + p * az)] = l[0][ax] * l[1][ay] * l[2][az];
}

static void node_of(const FmmBox& b, int p, const double* t, int n, double x[3]) {
  const int a[3] = {n % p, (n / p) % p, n / (p * p)};
  for (int d = 0; d < 3; ++d) x[d] = b.c[d] + b.h[d] * t[a[d]];
}

// ---- device ---------------------------------------------------------------------------

// M2L tensors of the far blocks [f0, f0 + nq): out[k * stride + (f - f0) * np3^2 + m * np3 + n]
// = exp(-sigma_k r) / (4 pi r), r = |x_n^X - y_m^Y| (column-major np3 x np3 slices)
template <typename T>
__global__ void __launch_bounds__(256) fmm_m2l_entries(const int2* __restrict__ fxy, int f0, int nq,
                                                       const double* __restrict__ box,
                                                       const double* __restrict__ tn, int p,
                                                       const double2* __restrict__ sig, int nK,
                                                       cpx<T>* __restrict__ out, int64_t stride) {
  const int np3 = p * p * p, ne = np3 * np3;
  for (int q = blockIdx.x; q < nq; q += gridDim.x) {
    const int2 xy = fxy[f0 + q];
    const double* bx = box + 6 * xy.x;
    const double* by = box + 6 * xy.y;
    for (int e = threadIdx.x; e < ne; e += blockDim.x) {
      const int n = e % np3, m = e / np3;
      const int an[3] = {n % p, (n / p) % p, n / (p * p)};
      const int am[3] = {m % p, (m / p) % p, m / (p * p)};
      double r2 = 0.0;
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const double dd = (bx[d] + bx[3 + d] * tn[an[d]]) - (by[d] + by[3 + d] * tn[am[d]]);
        r2 += dd * dd;
      }
      const double r = sqrt(r2);
      const double inv = INV4PI / r;
      cpx<T>* o = out + int64_t(q) * ne + e;
      for (int k = 0; k < nK; ++k) {
        const double2 sg = sig[k];
        const double a = exp(-sg.x * r) * inv;
        double sn, cs;
        sincos(sg.y * r, &sn, &cs);
        o[int64_t(k) * stride] = {T(a * cs), T(-a * sn)};
      }
    }
  }
}

// Xp[p][k] = X[k][perm[p]] (conjugated for conjugate-represented columns)
template <typename T>
__global__ void fmm_x_in(const cpx<T>* __restrict__ X, cpx<T>* __restrict__ Xp, const int* __restrict__ perm,
                         const int* __restrict__ conjflag, int n, int L) {
  const int64_t total = int64_t(n) * L;
  for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < total; e += int64_t(gridDim.x) * blockDim.x) {
    const int p = int(e / L), k = int(e % L);
    const cpx<T> x = X[int64_t(k) * n + perm[p]];
    Xp[e] = {x.re, conjflag[k] ? -x.im : x.im};
  }
}

// P2M: W[c][m][k] = sum_{p in leaf c} R[p][m] Xp[p][k]
template <typename T>
__global__ void __launch_bounds__(256) fmm_p2m(const int* __restrict__ leaves, int nleaves,
                                               const int* __restrict__ clbeg, const int* __restrict__ clend,
                                               const T* __restrict__ R, const cpx<T>* __restrict__ Xp,
                                               cpx<T>* __restrict__ W, int np3, int L) {
  for (int q = blockIdx.x; q < nleaves; q += gridDim.x) {
    const int c = leaves[q], b = clbeg[c], e1 = clend[c];
    for (int e = threadIdx.x; e < np3 * L; e += blockDim.x) {
      const int m = e / L, k = e % L;
      cpx<T> acc = {T(0), T(0)};
      for (int pp = b; pp < e1; ++pp) {
        const T r = R[int64_t(pp) * np3 + m];
        const cpx<T> x = Xp[int64_t(pp) * L + k];
        acc.re += r * x.re;
        acc.im += r * x.im;
      }
      W[(int64_t(c) * np3 + m) * L + k] = acc;
    }
  }
}

// M2M of one level: W[c][m'][k] = sum over the sons s of sum_m T[s][m][m'] W[s][m][k]
template <typename T>
__global__ void __launch_bounds__(256) fmm_m2m(const int* __restrict__ list, int cnt, const int* __restrict__ son0,
                                               const int* __restrict__ son1, const T* __restrict__ Tr,
                                               cpx<T>* __restrict__ W, int np3, int L) {
  for (int q = blockIdx.x; q < cnt; q += gridDim.x) {
    const int c = list[q];
    const int s[2] = {son0[c], son1[c]};
    for (int e = threadIdx.x; e < np3 * L; e += blockDim.x) {
      const int mp = e / L, k = e % L;
      cpx<T> acc = {T(0), T(0)};
      for (int h = 0; h < 2; ++h) {
        const T* ts = Tr + int64_t(s[h]) * np3 * np3;
        const cpx<T>* ws = W + int64_t(s[h]) * np3 * L + k;
        for (int m = 0; m < np3; ++m) {
          const T t = ts[int64_t(m) * np3 + mp];
          const cpx<T> w = ws[int64_t(m) * L];
          acc.re += t * w.re;
          acc.im += t * w.im;
        }
      }
      W[(int64_t(c) * np3 + mp) * L + k] = acc;
    }
  }
}

// M2L: per item (row cluster X, rows r0 .. r0 + FMM_RC of its local expansion)
// Z[X][n][k] = sum over the far blocks (X, Y) of sum_d f_d[kpos(k)] sum_m H_d[n][m] W[Y][m][k];
// the item's rows of each slice are staged in LDS
struct FmmItem {
  int X, r0, b0, nb;   // row cluster, first row, its far blocks rowlist[b0 .. b0 + nb)
};

template <typename T>
__global__ void __launch_bounds__(256) fmm_m2l(const FmmItem* __restrict__ items, int nitems,
                                               const int* __restrict__ rowlist, const int* __restrict__ fcol,
                                               const int* __restrict__ fstart, const int64_t* __restrict__ fslice,
                                               const int64_t* __restrict__ ffiber, const cpx<T>* __restrict__ pool,
                                               const int* __restrict__ kpos, const cpx<T>* __restrict__ W,
                                               cpx<T>* __restrict__ Z, int np3, int L) {
  __shared__ cpx<T> hs[FMM_RC * FMM_PMAX * FMM_PMAX * FMM_PMAX];
  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    const FmmItem I = items[it];
    const int nr = min(FMM_RC, np3 - I.r0);
    for (int k0 = 0; k0 < L; k0 += blockDim.x) {
      const int k = k0 + threadIdx.x;
      const bool kin = k < L;
      const int kp = kin ? kpos[k] : 0;
      cpx<T> z[FMM_RC];
#pragma unroll
      for (int r = 0; r < FMM_RC; ++r) z[r] = {T(0), T(0)};
      for (int bi = 0; bi < I.nb; ++bi) {
        const int f = rowlist[I.b0 + bi];
        const cpx<T>* wy = W + int64_t(fcol[f]) * np3 * L + (kin ? k : 0);
        for (int d = fstart[f]; d < fstart[f + 1]; ++d) {
          const cpx<T>* H = pool + fslice[d];
          __syncthreads();
          for (int e = threadIdx.x; e < nr * np3; e += blockDim.x) {
            const int r = e % nr, m = e / nr;
            hs[r * np3 + m] = H[int64_t(m) * np3 + I.r0 + r];
          }
          __syncthreads();
          cpx<T> acc[FMM_RC];
#pragma unroll
          for (int r = 0; r < FMM_RC; ++r) acc[r] = {T(0), T(0)};
          for (int m = 0; m < np3; ++m) {
            const cpx<T> w = wy[int64_t(m) * L];
#pragma unroll
            for (int r = 0; r < FMM_RC; ++r) {
              if (r >= nr) break;
              const cpx<T> h = hs[r * np3 + m];
              acc[r].re += h.re * w.re - h.im * w.im;
              acc[r].im += h.re * w.im + h.im * w.re;
            }
          }
          const cpx<T> fk = kin ? pool[ffiber[d] + kp] : cpx<T>{T(0), T(0)};
#pragma unroll
          for (int r = 0; r < FMM_RC; ++r) {
            z[r].re += fk.re * acc[r].re - fk.im * acc[r].im;
            z[r].im += fk.re * acc[r].im + fk.im * acc[r].re;
          }
        }
      }
      if (kin)
        for (int r = 0; r < nr; ++r) Z[(int64_t(I.X) * np3 + I.r0 + r) * L + k] = z[r];
    }
  }
}

// zero the local expansions of the clusters that receive no M2L term
template <typename T>
__global__ void fmm_zero(const int* __restrict__ list, int cnt, cpx<T>* __restrict__ Z, int np3, int L) {
  for (int q = blockIdx.x; q < cnt; q += gridDim.x) {
    cpx<T>* z = Z + int64_t(list[q]) * np3 * L;
    for (int e = threadIdx.x; e < np3 * L; e += blockDim.x) z[e] = {T(0), T(0)};
  }
}

// L2L of one level: Z[c][m][k] += sum_m' T[c][m][m'] Z[parent(c)][m'][k]
template <typename T>
__global__ void __launch_bounds__(256) fmm_l2l(const int* __restrict__ list, int cnt, const int* __restrict__ parent,
                                               const T* __restrict__ Tr, cpx<T>* __restrict__ Z, int np3, int L) {
  for (int q = blockIdx.x; q < cnt; q += gridDim.x) {
    const int c = list[q], P = parent[c];
    const T* tc = Tr + int64_t(c) * np3 * np3;
    const cpx<T>* zp = Z + int64_t(P) * np3 * L;
    for (int e = threadIdx.x; e < np3 * L; e += blockDim.x) {
      const int m = e / L, k = e % L;
      cpx<T> acc = Z[(int64_t(c) * np3 + m) * L + k];
      for (int mp = 0; mp < np3; ++mp) {
        const T t = tc[int64_t(m) * np3 + mp];
        const cpx<T> z = zp[int64_t(mp) * L + k];
        acc.re += t * z.re;
        acc.im += t * z.im;
      }
      Z[(int64_t(c) * np3 + m) * L + k] = acc;
    }
  }
}

// L2P and the output: Y[k][perm[p]] += sum_n L[p][n] Z[leaf(p)][n][k]
// (conjugated for conjugate-represented columns)
template <typename T>
__global__ void __launch_bounds__(256) fmm_l2p(const int* __restrict__ leaves, int nleaves,
                                               const int* __restrict__ clbeg, const int* __restrict__ clend,
                                               const T* __restrict__ Lx, const cpx<T>* __restrict__ Z,
                                               const int* __restrict__ perm, const int* __restrict__ conjflag,
                                               cpx<T>* __restrict__ Y, int n, int np3, int L) {
  for (int q = blockIdx.x; q < nleaves; q += gridDim.x) {
    const int c = leaves[q], b = clbeg[c], e1 = clend[c];
    const cpx<T>* zc = Z + int64_t(c) * np3 * L;
    for (int e = threadIdx.x; e < (e1 - b) * L; e += blockDim.x) {
      const int pp = b + e / L, k = e % L;
      cpx<T> acc = {T(0), T(0)};
      for (int nn = 0; nn < np3; ++nn) {
        const T l = Lx[int64_t(pp) * np3 + nn];
        const cpx<T> z = zc[int64_t(nn) * L + k];
        acc.re += l * z.re;
        acc.im += l * z.im;
      }
      cpx<T>* y = Y + int64_t(k) * n + perm[pp];
      const cpx<T> y0 = *y;
      *y = {y0.re + acc.re, y0.im + (conjflag[k] ? -acc.im : acc.im)};
    }
  }
}

static __global__ void fmm_zero_int(int* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

// ---- host tables of the product ---------------------------------------------------------

template <typename T>
static int fmm_tables(gcq_context* ctx, Fmm3D& M, const std::vector<FmmBox>& boxes, const double* t) {
  const int p = M.p, np3 = M.np3, n = ctx->n, nc = int(ctx->clusters.size());
  double rb[7][3], rw[7];
  radon7(rb, rw);
  std::vector<T> R(size_t(n) * np3, T(0)), Lx(size_t(n) * np3), Tr(size_t(nc) * np3 * np3, T(0));
  std::vector<double> row(np3);
  for (int c = 0; c < nc; ++c) {
    const Cluster& C = ctx->clusters[c];
    if (C.son0 >= 0) continue;
    for (int pp = C.begin; pp < C.end; ++pp) {
      const int tr = ctx->perm[pp];
      const double* v = &ctx->vert[9 * size_t(tr)];
      std::vector<double> acc(np3, 0.0);
      for (int q = 0; q < 7; ++q) {
        double y[3];
        for (int d = 0; d < 3; ++d) y[d] = rb[q][0] * v[d] + rb[q][1] * v[3 + d] + rb[q][2] * v[6 + d];
        interp_row(boxes[c], p, t, y, row.data());
        const double w = rw[q] * ctx->area[tr];
        for (int m = 0; m < np3; ++m) acc[m] += w * row[m];
      }
      for (int m = 0; m < np3; ++m) R[size_t(pp) * np3 + m] = T(acc[m]);
      interp_row(boxes[c], p, t, &ctx->cen[3 * size_t(tr)], row.data());
      for (int m = 0; m < np3; ++m) Lx[size_t(pp) * np3 + m] = T(row[m]);
    }
  }
  for (int c = 0; c < nc; ++c) {
    const Cluster& C = ctx->clusters[c];
    for (int h = 0; h < 2; ++h) {
      const int s = h == 0 ? C.son0 : C.son1;
      if (s < 0) continue;
      for (int m = 0; m < np3; ++m) {
        double y[3];
        node_of(boxes[s], p, t, m, y);
        interp_row(boxes[c], p, t, y, row.data());
        for (int mp = 0; mp < np3; ++mp) Tr[(size_t(s) * np3 + m) * np3 + mp] = T(row[mp]);
      }
    }
  }
  GCQ_TRY(upload(M.d_R, R, ctx->stream));
  GCQ_TRY(upload(M.d_L, Lx, ctx->stream));
  GCQ_TRY(upload(M.d_T, Tr, ctx->stream));
  GCQ_HIP(hipStreamSynchronize(ctx->stream));
  M.table_bytes = int64_t(R.size() + Lx.size() + Tr.size()) * int64_t(sizeof(T));
  return GCQ_OK;
}

template <typename T>
static void fmm_far_product(gcq_context* ctx, const void* X, void* Y) {
  Fmm3D& M = ctx->Mf;
  const int n = ctx->n, L = ctx->L, np3 = M.np3;
  hipStream_t st = ctx->stream;
  cpx<T>* Xp = M.Xp.as<cpx<T>>();
  cpx<T>* W = M.W.as<cpx<T>>();
  cpx<T>* Z = M.Z.as<cpx<T>>();
  const int* conjf = M.d_conj.as<int>();
  const int grid = ctx->cus * 4;
  hipLaunchKernelGGL(fmm_x_in<T>, dim3(4096), dim3(256), 0, st, static_cast<const cpx<T>*>(X), Xp,
                     ctx->d_perm.as<int>(), conjf, n, L);
  hipLaunchKernelGGL(fmm_p2m<T>, dim3(std::min(M.nleaves, grid)), dim3(256), 0, st, M.d_leaves.as<int>(), M.nleaves,
                     M.d_clbeg.as<int>(), M.d_clend.as<int>(), M.d_R.as<T>(), Xp, W, np3, L);
  // upward: levels from the deepest, clusters with sons
  for (int lev = int(M.lev_start.size()) - 2; lev >= 0; --lev) {
    const int c0 = M.lev_start[lev], cnt = M.lev_start[lev + 1] - c0;
    if (cnt > 0)
      hipLaunchKernelGGL(fmm_m2m<T>, dim3(std::min(cnt, grid)), dim3(256), 0, st, M.d_uplist.as<int>() + c0, cnt,
                         M.d_son0.as<int>(), M.d_son1.as<int>(), M.d_T.as<T>(), W, np3, L);
  }
  if (M.nzero > 0)
    hipLaunchKernelGGL(fmm_zero<T>, dim3(std::min(M.nzero, grid)), dim3(256), 0, st, M.d_zlist.as<int>(), M.nzero,
                       Z, np3, L);
  if (M.nitems > 0)
    hipLaunchKernelGGL(fmm_m2l<T>, dim3(std::min(M.nitems, grid * 2)), dim3(256), 0, st, M.d_items.as<FmmItem>(),
                       M.nitems, M.d_rowlist.as<int>(), M.d_fcol.as<int>(), M.d_fstart.as<int>(),
                       M.d_fslice.as<int64_t>(), M.d_ffiber.as<int64_t>(), M.pool.as<cpx<T>>(),
                       M.d_kpos.as<int>(), W, Z, np3, L);
  // downward: depth 1 onwards
  for (size_t lev = 1; lev + 1 < M.down_start.size(); ++lev) {
    const int c0 = M.down_start[lev], cnt = M.down_start[lev + 1] - c0;
    if (cnt > 0)
      hipLaunchKernelGGL(fmm_l2l<T>, dim3(std::min(cnt, grid)), dim3(256), 0, st, M.d_downlist.as<int>() + c0, cnt,
                         M.d_parent.as<int>(), M.d_T.as<T>(), Z, np3, L);
  }
  hipLaunchKernelGGL(fmm_l2p<T>, dim3(std::min(M.nleaves, grid)), dim3(256), 0, st, M.d_leaves.as<int>(),
                     M.nleaves, M.d_clbeg.as<int>(), M.d_clend.as<int>(), M.d_L.as<T>(), Z, ctx->d_perm.as<int>(),
                     conjf, static_cast<cpx<T>*>(Y), n, np3, L);
}

}  // namespace gcq

using namespace gcq;

extern "C" GCQ_API int gcq_fmm3d(gcq_context* ctx, int32_t order, double tol, int32_t max_freq_rank,
                                 int32_t precision, gcq_fmm3d_stats* stats) {
  if (!ctx) return fail(GCQ_ERR_ARG, "ctx is NULL");
  GCQ_NEED_DEVICE(ctx);
  if (!ctx->have_tree || !ctx->have_freq)
    return fail(GCQ_ERR_STATE, "upload mesh, frequencies and build the tree first");
  if (order < 1 || order > FMM_PMAX) return fail(GCQ_ERR_ARG, "order must be in 1..%d", FMM_PMAX);
  if (precision != GCQ_C128 && precision != GCQ_C64) return fail(GCQ_ERR_ARG, "unknown precision %d", precision);
  if (!(tol >= 0.0)) return fail(GCQ_ERR_ARG, "tol must be >= 0");
  if (max_freq_rank < 1 || max_freq_rank > R3_MAX)
    return fail(GCQ_ERR_ARG, "max_freq_rank must be in 1..%d", R3_MAX);
  Fmm3D& M = ctx->Mf;
  M.valid = false;
  // near field: the 3D-ACA of the inadmissible blocks (dense slices)
  gcq_aca3d_stats nst;
  GCQ_TRY(aca3d_run(ctx, 0.0, tol, max_freq_rank, precision, 0u, true, &nst));
  GCQ_HIP(hipSetDevice(ctx->device));
  const int p = order, np3 = p * p * p, nK = int(ctx->K.size()), L = ctx->L, n = ctx->n;
  const int nc = int(ctx->clusters.size());
  const int64_t csz = csize(precision);
  hipStream_t st = ctx->stream;
  M.p = p;
  M.np3 = np3;
  M.precision = precision;
  M.nK = nK;
  double t[FMM_PMAX];
  cheb_nodes(p, t);
  std::vector<FmmBox> boxes(nc);
  std::vector<double> boxv(6 * size_t(nc));
  for (int c = 0; c < nc; ++c) {
    boxes[c] = box_of(ctx->clusters[c]);
    for (int d = 0; d < 3; ++d) {
      boxv[6 * c + d] = boxes[c].c[d];
      boxv[6 * c + 3 + d] = boxes[c].h[d];
    }
  }
  // far blocks
  const int nfar = int(ctx->far_ids.size());
  M.nfar = nfar;
  std::vector<int2> fxy(nfar);
  for (int f = 0; f < nfar; ++f) {
    const Block& B = ctx->blocks[ctx->far_ids[f]];
    fxy[f] = make_int2(B.row, B.col);
  }
  std::vector<double2> sig(nK);
  for (int q = 0; q < nK; ++q) {
    const std::complex<double> s = ctx->s[ctx->K[q]] / ctx->c;
    sig[q] = make_double2(s.real(), s.imag());
  }
  DevBuf d_box, d_t, d_sig, d_fxy, d_desc, d_ids, d_off, d_q, d_terms, d_rank, d_stat, d_cnt;
  GCQ_TRY(upload(d_box, boxv, st));
  GCQ_TRY(upload(d_t, std::vector<double>(t, t + p), st));
  GCQ_TRY(upload(d_sig, sig, st));
  GCQ_TRY(upload(d_fxy, fxy, st));
  std::vector<BlockDesc3> desc(std::max(nfar, 1), BlockDesc3{0, np3, 0, np3, 0, 0, 0, 0});
  std::vector<int> ids(std::max(nfar, 1));
  std::iota(ids.begin(), ids.end(), 0);
  std::vector<int64_t> off(std::max(nfar, 1));
  for (int f = 0; f < nfar; ++f) off[f] = int64_t(f) * np3 * np3;
  GCQ_TRY(upload(d_desc, desc, st));
  GCQ_TRY(upload(d_ids, ids, st));
  GCQ_TRY(upload(d_off, off, st));
  GCQ_TRY(d_q.ensure(sizeof(int) * size_t(std::max(nfar, 1))));
  GCQ_TRY(d_terms.ensure(sizeof(Term3) * size_t(std::max(nfar, 1)) * R3_MAX));
  GCQ_TRY(d_rank.ensure(sizeof(int) * 2 * size_t(std::max(nfar, 1))));
  GCQ_TRY(d_cnt.ensure(256));
  int* d_brank = d_rank.as<int>();
  int* d_bstat = d_brank + std::max(nfar, 1);
  unsigned long long* d_cursor = d_cnt.as<unsigned long long>();
  int* d_counter = reinterpret_cast<int*>(d_cnt.as<unsigned char>() + 64);
  hipLaunchKernelGGL(fmm_zero_int, dim3((2 * std::max(nfar, 1) + 63) / 64), dim3(64), 0, st, d_brank,
                     2 * std::max(nfar, 1));
  // pool: slices and fibers of the M2L terms
  size_t freeb = 0, totalb = 0;
  GCQ_HIP(hipMemGetInfo(&freeb, &totalb));
  const int64_t rexp = 8;
  int64_t capacity = std::max<int64_t>(int64_t(1) << 20, int64_t(nfar) * rexp * (int64_t(np3) * np3 + nK));
  capacity = std::min<int64_t>(capacity, int64_t(double(freeb) * 0.25) / csz);
  GCQ_TRY(M.pool.ensure(size_t(capacity) * csz + 256));
  const int64_t tensor_budget =
      std::max<int64_t>(int64_t(1) << 28, std::min<int64_t>(int64_t(16) << 30, int64_t(double(freeb) * 0.15)));
  const int64_t per_block = int64_t(np3) * np3 * nK * csz;
  const int batch = int(std::max<int64_t>(1, tensor_budget / per_block));
  DevBuf& tensor = ctx->scratchT;
  std::vector<int> todo(nfar), brank(std::max(nfar, 1)), bstat(std::max(nfar, 1));
  std::iota(todo.begin(), todo.end(), 0);
  int64_t used = 0;
  double ms = 0.0;
  for (int round = 0; round < 8 && !todo.empty(); ++round) {
    unsigned long long cur0 = (unsigned long long)used;
    GCQ_HIP(hipMemcpyAsync(d_cursor, &cur0, sizeof(cur0), hipMemcpyHostToDevice, st));
    GCQ_HIP(hipMemcpyAsync(d_q.p, todo.data(), sizeof(int) * todo.size(), hipMemcpyHostToDevice, st));
    GCQ_HIP(hipStreamSynchronize(st));
    // batches of consecutive entries of the to-do list (rounds after the first
    // redo the blocks the pool could not hold)
    for (size_t pos = 0; pos < todo.size();) {
      // the tensor of a batch covers far blocks [todo[pos], todo[end - 1]]
      size_t end = pos + 1;
      while (end < todo.size() && todo[end] - todo[pos] < batch) ++end;
      const int f0 = todo[pos], span_blocks = todo[end - 1] - f0 + 1;
      const int64_t stride = int64_t(span_blocks) * np3 * np3;
      GCQ_TRY(tensor.ensure(size_t(stride) * nK * csz + 256));
      GCQ_TRY(timed_begin(ctx));
      if (precision == GCQ_C128)
        hipLaunchKernelGGL(fmm_m2l_entries<double>, dim3(std::min(span_blocks, 65536)), dim3(256), 0, st,
                           d_fxy.as<int2>(), f0, span_blocks, d_box.as<double>(), d_t.as<double>(), p,
                           d_sig.as<double2>(), nK, tensor.as<cpx<double>>(), stride);
      else
        hipLaunchKernelGGL(fmm_m2l_entries<float>, dim3(std::min(span_blocks, 65536)), dim3(256), 0, st,
                           d_fxy.as<int2>(), f0, span_blocks, d_box.as<double>(), d_t.as<double>(), p,
                           d_sig.as<double2>(), nK, tensor.as<cpx<float>>(), stride);
      GCQ_HIP(hipGetLastError());
      hipLaunchKernelGGL(fmm_zero_int, dim3(1), dim3(64), 0, st, d_counter, 1);
      const int cnt = int(end - pos);
      launch_dense_aca3d(precision, std::min(cnt, ctx->cus * 16), st, d_desc.as<BlockDesc3>(),
                         d_q.as<int>() + pos, cnt, d_ids.as<int>(), d_off.as<int64_t>(), int64_t(f0) * np3 * np3,
                         tensor.p, stride, nK, tol, int(max_freq_rank), M.pool.p, d_cursor, capacity,
                         d_terms.as<Term3>(), d_brank, d_bstat, d_counter);
      GCQ_HIP(hipGetLastError());
      ms += timed_end(ctx, "fmm3d_m2l_batch");
      pos = end;
    }
    unsigned long long curh = 0;
    GCQ_HIP(hipMemcpy(&curh, d_cursor, sizeof(curh), hipMemcpyDeviceToHost));
    GCQ_HIP(hipMemcpy(brank.data(), d_brank, sizeof(int) * brank.size(), hipMemcpyDeviceToHost));
    GCQ_HIP(hipMemcpy(bstat.data(), d_bstat, sizeof(int) * bstat.size(), hipMemcpyDeviceToHost));
    used = std::min<int64_t>(int64_t(curh), capacity);
    std::vector<int> again;
    for (int f : todo)
      if (bstat[f] & ST_DEFERRED) again.push_back(f);
    if (!again.empty()) {
      const int64_t newcap = capacity * 2;
      DevBuf bigger;
      GCQ_TRY(bigger.ensure(size_t(newcap) * csz + 256));
      GCQ_HIP(hipMemcpy(bigger.p, M.pool.p, size_t(used) * csz, hipMemcpyDeviceToDevice));
      std::swap(bigger.p, M.pool.p);
      std::swap(bigger.bytes, M.pool.bytes);
      capacity = newcap;
    }
    todo.swap(again);
  }
  if (!todo.empty()) return fail(GCQ_ERR_NOMEM, "the M2L pool could not hold the result");
  tensor.release();
  // terms of every far block
  std::vector<Term3> terms(size_t(std::max(nfar, 1)) * R3_MAX);
  GCQ_HIP(hipMemcpy(terms.data(), d_terms.p, sizeof(Term3) * terms.size(), hipMemcpyDeviceToHost));
  M.fstart.assign(nfar + 1, 0);
  M.fslice.clear();
  M.ffiber.clear();
  M.ffreq.clear();
  int rmax_seen = 0, ncap = 0;
  int64_t words = 0;
  for (int f = 0; f < nfar; ++f) {
    M.fstart[f + 1] = M.fstart[f] + brank[f];
    rmax_seen = std::max(rmax_seen, brank[f]);
    ncap += (bstat[f] & ST_CAPPED) != 0;
    for (int d = 0; d < brank[f]; ++d) {
      const Term3& tm = terms[size_t(f) * R3_MAX + d];
      M.fslice.push_back(tm.slice);
      M.ffiber.push_back(tm.fiber);
      M.ffreq.push_back(tm.freq);
      words += int64_t(np3) * np3 + nK;
    }
  }
  // product tables: M2L items per row cluster, leaves, levels, interpolation
  std::vector<int> fcol(std::max(nfar, 1)), rowlist;
  std::vector<std::vector<int>> byrow(nc);
  for (int f = 0; f < nfar; ++f) {
    fcol[f] = fxy[f].y;
    if (brank[f] > 0) byrow[fxy[f].x].push_back(f);
  }
  std::vector<FmmItem> items;
  std::vector<int> zlist;
  for (int c = 0; c < nc; ++c) {
    if (byrow[c].empty()) {
      zlist.push_back(c);
      continue;
    }
    const int b0 = int(rowlist.size());
    rowlist.insert(rowlist.end(), byrow[c].begin(), byrow[c].end());
    for (int r0 = 0; r0 < np3; r0 += FMM_RC) items.push_back({c, r0, b0, int(byrow[c].size())});
  }
  // most work first
  std::stable_sort(items.begin(), items.end(), [](const FmmItem& a, const FmmItem& b) { return a.nb > b.nb; });
  std::vector<int> leaves, clbeg(nc), clend(nc), son0(nc), son1(nc), parent(nc, -1);
  int maxdepth = 0;
  for (int c = 0; c < nc; ++c) {
    const Cluster& C = ctx->clusters[c];
    clbeg[c] = C.begin;
    clend[c] = C.end;
    son0[c] = C.son0;
    son1[c] = C.son1;
    if (C.son0 >= 0) parent[C.son0] = c;
    if (C.son1 >= 0) parent[C.son1] = c;
    if (C.son0 < 0) leaves.push_back(c);
    maxdepth = std::max(maxdepth, C.depth);
  }
  // upward list: clusters with sons by depth; downward list: all but the root by depth
  std::vector<int> uplist, downlist;
  M.lev_start.assign(1, 0);
  M.down_start.assign(1, 0);
  for (int dep = 0; dep <= maxdepth; ++dep) {
    for (int c = 0; c < nc; ++c)
      if (ctx->clusters[c].depth == dep) {
        if (ctx->clusters[c].son0 >= 0) uplist.push_back(c);
        downlist.push_back(c);
      }
    M.lev_start.push_back(int(uplist.size()));
    M.down_start.push_back(int(downlist.size()));
  }
  std::vector<int> conjv(ctx->conj.begin(), ctx->conj.end()), kposv(ctx->kpos.begin(), ctx->kpos.end());
  GCQ_TRY(upload(M.d_fstart, M.fstart, st));
  GCQ_TRY(upload(M.d_fslice, M.fslice.empty() ? std::vector<int64_t>(1, 0) : M.fslice, st));
  GCQ_TRY(upload(M.d_ffiber, M.ffiber.empty() ? std::vector<int64_t>(1, 0) : M.ffiber, st));
  GCQ_TRY(upload(M.d_fcol, fcol, st));
  GCQ_TRY(upload(M.d_rowlist, rowlist.empty() ? std::vector<int>(1, 0) : rowlist, st));
  GCQ_TRY(upload(M.d_items, items.empty() ? std::vector<FmmItem>(1) : items, st));
  GCQ_TRY(upload(M.d_zlist, zlist.empty() ? std::vector<int>(1, 0) : zlist, st));
  GCQ_TRY(upload(M.d_leaves, leaves, st));
  GCQ_TRY(upload(M.d_clbeg, clbeg, st));
  GCQ_TRY(upload(M.d_clend, clend, st));
  GCQ_TRY(upload(M.d_son0, son0, st));
  GCQ_TRY(upload(M.d_son1, son1, st));
  GCQ_TRY(upload(M.d_parent, parent, st));
  GCQ_TRY(upload(M.d_uplist, uplist.empty() ? std::vector<int>(1, 0) : uplist, st));
  GCQ_TRY(upload(M.d_downlist, downlist, st));
  GCQ_TRY(upload(M.d_conj, conjv, st));
  GCQ_TRY(upload(M.d_kpos, kposv, st));
  GCQ_HIP(hipStreamSynchronize(st));
  M.nitems = int(items.size());
  M.nzero = int(zlist.size());
  M.nleaves = int(leaves.size());
  if (precision == GCQ_C128)
    GCQ_TRY(fmm_tables<double>(ctx, M, boxes, t));
  else
    GCQ_TRY(fmm_tables<float>(ctx, M, boxes, t));
  M.m2l_bytes = words * csz;
  M.valid = true;
  ctx->kernel_ms["fmm3d_m2l"] = ms;
  if (stats) {
    int64_t rs = 0;
    for (int f = 0; f < nfar; ++f) rs += brank[f];
    stats->n_far = nfar;
    stats->rank_max = rmax_seen;
    stats->rank_mean = nfar > 0 ? double(rs) / nfar : 0.0;
    stats->n_capped = ncap;
    stats->storage_bytes = M.m2l_bytes + M.table_bytes + nst.storage_bytes;
    stats->device_ms = ms + nst.device_ms;
    stats->m2l_ms = ms;
  }
  return GCQ_OK;
}

extern "C" GCQ_API int gcq_fmm3d_matvec(gcq_context* ctx, const void* X_dev, void* Y_dev) {
  if (!ctx) return fail(GCQ_ERR_ARG, "ctx is NULL");
  GCQ_NEED_DEVICE(ctx);
  Fmm3D& M = ctx->Mf;
  if (!M.valid || !ctx->F.valid || !ctx->F.near_only) return fail(GCQ_ERR_STATE, "run gcq_fmm3d first");
  GCQ_HIP(hipSetDevice(ctx->device));
  GCQ_TRY(check_device_ptr(ctx, X_dev, "X_dev"));
  GCQ_TRY(check_device_ptr(ctx, Y_dev, "Y_dev"));
  const int64_t csz = csize(M.precision);
  const size_t nc = ctx->clusters.size();
  GCQ_TRY(M.Xp.ensure(size_t(ctx->n) * ctx->L * csz + 256));
  GCQ_TRY(M.W.ensure(nc * M.np3 * ctx->L * csz + 256));
  GCQ_TRY(M.Z.ensure(nc * M.np3 * ctx->L * csz + 256));
  // near field into Y, then the far field added
  GCQ_TRY(run_compressed(ctx, GCQ_PER_FREQUENCY, M.precision, X_dev, Y_dev));
  GCQ_TRY(timed_begin(ctx));
  if (M.precision == GCQ_C128)
    fmm_far_product<double>(ctx, X_dev, Y_dev);
  else
    fmm_far_product<float>(ctx, X_dev, Y_dev);
  GCQ_HIP(hipGetLastError());
  ctx->kernel_ms["fmm3d_far"] = timed_end(ctx, "fmm3d_far");
  GCQ_HIP(hipStreamSynchronize(ctx->stream));
  return GCQ_OK;
}

extern "C" GCQ_API int gcq_get_fmm3d_block(gcq_context* ctx, int32_t block, int32_t cap, int32_t* rank,
                                           int32_t* freqs, gcq_c128* fibers, gcq_c128* slices) {
  if (!ctx) return fail(GCQ_ERR_ARG, "ctx is NULL");
  const Fmm3D& M = ctx->Mf;
  if (!M.valid) return fail(GCQ_ERR_STATE, "run gcq_fmm3d first");
  if (!rank) return fail(GCQ_ERR_ARG, "rank is NULL");
  const int f = int(std::lower_bound(ctx->far_ids.begin(), ctx->far_ids.end(), block) - ctx->far_ids.begin());
  if (block < 0 || f >= int(ctx->far_ids.size()) || ctx->far_ids[f] != block)
    return fail(GCQ_ERR_ARG, "block %d is not an admissible block", block);
  const int r = M.fstart[f + 1] - M.fstart[f];
  *rank = r;
  if (r > cap) return fail(GCQ_ERR_ARG, "rank %d exceeds cap %d", r, cap);
  const int64_t ne = int64_t(M.np3) * M.np3;
  for (int d = 0; d < r; ++d) {
    const int ti = M.fstart[f] + d;
    if (freqs) freqs[d] = M.ffreq[ti];
    auto fetch = [&](int64_t off, int64_t cnt, gcq_c128* out) -> int {
      if (M.precision == GCQ_C128) {
        GCQ_HIP(hipMemcpy(out, M.pool.as<cpx<double>>() + off, cnt * 16, hipMemcpyDeviceToHost));
      } else {
        std::vector<cpx<float>> tmp(cnt);
        GCQ_HIP(hipMemcpy(tmp.data(), M.pool.as<cpx<float>>() + off, cnt * 8, hipMemcpyDeviceToHost));
        for (int64_t e = 0; e < cnt; ++e) out[e] = {tmp[e].re, tmp[e].im};
      }
      return GCQ_OK;
    };
    if (fibers) GCQ_TRY(fetch(M.ffiber[ti], M.nK, fibers + int64_t(d) * M.nK));
    if (slices) GCQ_TRY(fetch(M.fslice[ti], ne, slices + int64_t(d) * ne));
  }
  return GCQ_OK;
}
