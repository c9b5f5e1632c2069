// Dense near-field blocks at many frequencies at once.
//
// The entries of every inadmissible block are written for F frequencies into
// out[f * stride + near_off[q] + e] (e column-major inside the block).  Two
// passes keep the waves uniform:
//   near_far_tier: one thread per entry; entries of the far tier (7-point rule,
//     in T) evaluate their 7 distances once and loop over the frequencies;
//     self and near-tier entries are skipped;
//   near_sing: one thread per (self/near-tier entry, frequency), float64
//     (polar-coordinate self rule or 112-point rule).
// DLP: the double layer's entries (normal derivative in y; self entries 0).
// The list of self/near-tier entries is built once with the block tree.
#pragma once
#include "device_common.h"

namespace gcq {

struct SingEntry {
  int64_t off;   // element offset inside one frequency's near storage
  int pi, pj;    // internal positions
};

template <typename T, bool DLP = false>
__global__ void __launch_bounds__(256) near_far_tier(Tab tab, const int* __restrict__ blk,
                                                     const int* __restrict__ near_ids,
                                                     const int64_t* __restrict__ near_off,
                                                     int q0, int q1, int64_t base0,
                                                     const double2* __restrict__ sig, int F,
                                                     cpx<T>* __restrict__ out, int64_t stride) {
  for (int q = q0 + blockIdx.x; q < q1; q += gridDim.x) {
    const int id = near_ids[q];
    const int rb = blk[5 * id], m = blk[5 * id + 1] - rb, cb = blk[5 * id + 2];
    const int n = blk[5 * id + 3] - cb;
    const int64_t base = near_off[q] - base0;
    for (int e = threadIdx.x; e < m * n; e += blockDim.x) {
      const int r = e % m, c = e / m;
      const int pi = rb + r, pj = cb + c;
      if (pi == pj || is_near(tab, pi, pj)) continue;
      const T* cen = FarData<T>::c(tab);
      const T* qp = FarData<T>::q(tab);
      const int nn = tab.n;
      const T xi = cen[pi], yi = cen[nn + pi], zi = cen[2 * nn + pi];
      T rr[NQ_FAR], ww[NQ_FAR];
      T nrm[3] = {T(0), T(0), T(0)};
      if constexpr (DLP) panel_normal(tab, pj, nrm);
#pragma unroll
      for (int a = 0; a < NQ_FAR; ++a) {
        const T dx = xi - qp[a * nn + pj], dy = yi - qp[(7 + a) * nn + pj];
        const T dz = zi - qp[(14 + a) * nn + pj];
        const T r2 = dx * dx + dy * dy + dz * dz;
        rr[a] = sqrt(r2);
        ww[a] = qp[(21 + a) * nn + pj];
        if constexpr (DLP) ww[a] *= (dx * nrm[0] + dy * nrm[1] + dz * nrm[2]) / (r2 * rr[a]);
      }
      for (int f = 0; f < F; ++f) {
        const double2 s = sig[f];
        cpx<T> acc = {T(0), T(0)};
#pragma unroll
        for (int a = 0; a < NQ_FAR; ++a) {
          const cpx<T> gg = DLP ? dlp_radial(rr[a], T(s.x), T(s.y)) : green(rr[a], T(s.x), T(s.y));
          acc.re += ww[a] * gg.re;
          acc.im += ww[a] * gg.im;
        }
        out[int64_t(f) * stride + base + e] = acc;
      }
    }
  }
}

template <typename T, bool DLP = false>
__global__ void __launch_bounds__(256) near_sing(Tab tab, const SingEntry* __restrict__ list,
                                                 int64_t s0, int64_t s1, int64_t base0,
                                                 const double2* __restrict__ sig, int F,
                                                 cpx<T>* __restrict__ out, int64_t stride) {
  const int64_t total = (s1 - s0) * F;
  for (int64_t x = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; x < total;
       x += int64_t(gridDim.x) * blockDim.x) {
    const int64_t a = s0 + x / F;
    const int f = int(x % F);
    const SingEntry se = list[a];
    const double2 s = sig[f];
    cpx<double> v;
    if constexpr (DLP)
      v = se.pi == se.pj ? cpx<double>{0.0, 0.0} : dlp_near_entry(tab, se.pi, se.pj, s.x, s.y);
    else
      v = se.pi == se.pj ? self_entry(tab, se.pi, s.x, s.y) : near_entry(tab, se.pi, se.pj, s.x, s.y);
    out[int64_t(f) * stride + se.off - base0] = {T(v.re), T(v.im)};
  }
}

}  // namespace gcq
