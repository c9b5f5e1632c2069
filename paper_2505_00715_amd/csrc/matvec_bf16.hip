// Per-frequency product with the 3D-ACA form (eq. product) on the bf16 matrix
// cores of gfx950 with float accumulation (v_mfma_f32_32x32x16_bf16), float
// operands split into bf16 planes:
//   operator a = ha + la + ra,            ha = bf16(a), la = bf16(a - ha),
//                                         |ra| <= 2^-18 |a| (dropped: a fixed
//                                         perturbation of the operator)
//   vector   x = hx + mx + lx + rx,       mx = bf16(x - hx), lx = bf16(x - hx - mx),
//                                         |rx| <= 2^-27 |x|
//   a x ~ ha hx + ha mx + ha lx + la hx + la mx          (la lx <= 2^-27 |a x| dropped)
// so the computed product is (a - ra) x up to 2^-26 |a| |x|: linear in x to
// about float rounding, which a Krylov solver needs (two planes for x as well
// would leave a part of 2^-17 that depends on the rounding of x and stalls
// GMRES near 1e-5).  A complex product takes four real ones (Re = rr - ii,
// Im = ri + ir), so one complex multiply-add costs 20 bf16 products, against 3
// float products (Gauss) on the float matrix cores, which run at 1/16 of the
// bf16 rate.
//
// Operand storage: "groups" of 8 consecutive values along the contraction
// index, holding the planes of those 8 values (operator groups: hi(Re), lo(Re),
// hi(Im), lo(Im), 64 bytes; vector groups: hi, mid, lo of Re then of Im, 96
// bytes).  Contractions over a block's columns (Vbar^H X_J, D_d X_J) use
// groups aligned to global cluster positions (group g covers positions
// 8g .. 8g + 7), so the slice groups and the right-hand side's groups line up
// and every lane load is an aligned 16-byte load; positions outside the block
// are zero in the slice groups.
//   far block (R stacked columns): Vg[c][g] = conj(Vbar[:, c]) over the
//     block's column groups; Ug[i][gc] = Ubar[i, 8 gc .. 8 gc + 7]
//   near block, term d: Dg_d[i][g] = D_d[i, :] over the column groups
//   right-hand side: Xg[k][g] (frequency k, all positions of the mesh)
// The product: per block and 64-column chunk of frequencies, as in the float
// kernel -- far: T = Vbar^H X_J (stacked columns x 64), T' = F o T (fibers),
// split into vector planes in LDS, Y_I += Ubar T'; near:
// Y_I += sum_d f_d o (D_d X_J); float atomics into Y (frequency fastest),
// permuted out afterwards.
#include <algorithm>
#include <cstring>
#include <numeric>
#include <vector>

#include "internal.h"
#include "matvec.h"

namespace gcq {

typedef __bf16 bf8v __attribute__((ext_vector_type(8)));
typedef float f16v __attribute__((ext_vector_type(16)));

struct alignas(16) BfGroup {
  uint4 hr, lr, hi, li;   // operator: 8 bf16 each, hi/lo planes of Re and Im
};
static_assert(sizeof(BfGroup) == 64, "group of 8 values in four planes");
struct alignas(16) BfGroup3 {
  uint4 hr, mr, lr, hi, mi, li;   // vector: hi/mid/lo planes of Re, then of Im
};
static_assert(sizeof(BfGroup3) == 96, "group of 8 values in six planes");

__device__ __forceinline__ unsigned short bf_bits(__bf16 h) { return __builtin_bit_cast(unsigned short, h); }

// hi = bf16(x) (round to nearest even), lo = bf16(x - hi)
__device__ __forceinline__ void split1(float x, unsigned short& h, unsigned short& l) {
  const __bf16 hb = static_cast<__bf16>(x);
  const __bf16 lb = static_cast<__bf16>(x - static_cast<float>(hb));
  h = bf_bits(hb);
  l = bf_bits(lb);
}

// x = hi + mid + lo (+ <= 2^-27 |x|)
__device__ __forceinline__ void split3(float x, unsigned short& h, unsigned short& m, unsigned short& l) {
  const __bf16 hb = static_cast<__bf16>(x);
  const float r1 = x - static_cast<float>(hb);
  const __bf16 mb = static_cast<__bf16>(r1);
  const __bf16 lb = static_cast<__bf16>(r1 - static_cast<float>(mb));
  h = bf_bits(hb);
  m = bf_bits(mb);
  l = bf_bits(lb);
}

__device__ __forceinline__ uint4 pack8(const unsigned short* s) {
  return make_uint4(s[0] | (unsigned(s[1]) << 16), s[2] | (unsigned(s[3]) << 16),
                    s[4] | (unsigned(s[5]) << 16), s[6] | (unsigned(s[7]) << 16));
}

// 8 complex values into a vector group
__device__ __forceinline__ BfGroup3 make_group3(const cpx<float>* v) {
  unsigned short hr[8], mr[8], lr[8], hi[8], mi[8], li[8];
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    split3(v[e].re, hr[e], mr[e], lr[e]);
    split3(v[e].im, hi[e], mi[e], li[e]);
  }
  BfGroup3 g;
  g.hr = pack8(hr);
  g.mr = pack8(mr);
  g.lr = pack8(lr);
  g.hi = pack8(hi);
  g.mi = pack8(mi);
  g.li = pack8(li);
  return g;
}

// 8 complex values into an operator group
__device__ __forceinline__ BfGroup make_group(const cpx<float>* v) {
  unsigned short hr[8], lr[8], hi[8], li[8];
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    split1(v[e].re, hr[e], lr[e]);
    split1(v[e].im, hi[e], li[e]);
  }
  BfGroup g;
  auto pack = [](const unsigned short* s) {
    return make_uint4(s[0] | (unsigned(s[1]) << 16), s[2] | (unsigned(s[3]) << 16),
                      s[4] | (unsigned(s[5]) << 16), s[6] | (unsigned(s[7]) << 16));
  };
  g.hr = pack(hr);
  g.lr = pack(lr);
  g.hi = pack(hi);
  g.li = pack(li);
  return g;
}

__device__ __forceinline__ bf8v as_bf8(uint4 u) { return __builtin_bit_cast(bf8v, u); }

__device__ __forceinline__ f16v f16_zero() {
  f16v z;
#pragma unroll
  for (int r = 0; r < 16; ++r) z[r] = 0.f;
  return z;
}

__device__ __forceinline__ f16v mf(uint4 a, uint4 b, f16v c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(as_bf8(a), as_bf8(b), c, 0, 0, 0);
}

// one real product of an operator part (hi, lo) and a vector part (hi, mid,
// lo): ha hx + ha mx + ha lx + la hx + la mx
__device__ __forceinline__ f16v rprod(uint4 ah, uint4 al, uint4 xh, uint4 xm, uint4 xl, f16v c) {
  c = mf(ah, xh, c);
  c = mf(ah, xm, c);
  c = mf(ah, xl, c);
  c = mf(al, xh, c);
  c = mf(al, xm, c);
  return c;
}

// one contraction step of 16 complex values (two groups per lane pair):
// rr += Re a Re x, ii += Im a Im x, ri += Re a Im x + Im a Re x
__device__ __forceinline__ void cstep(const BfGroup& a, const BfGroup3& x, f16v& rr, f16v& ii, f16v& ri) {
  rr = rprod(a.hr, a.lr, x.hr, x.mr, x.lr, rr);
  ii = rprod(a.hi, a.li, x.hi, x.mi, x.li, ii);
  ri = rprod(a.hr, a.lr, x.hi, x.mi, x.li, ri);
  ri = rprod(a.hi, a.li, x.hr, x.mr, x.lr, ri);
}

__device__ __forceinline__ BfGroup zero_group() {
  BfGroup g;
  g.hr = g.lr = g.hi = g.li = make_uint4(0, 0, 0, 0);
  return g;
}
__device__ __forceinline__ BfGroup3 zero_group3() {
  BfGroup3 g;
  g.hr = g.mr = g.lr = g.hi = g.mi = g.li = make_uint4(0, 0, 0, 0);
  return g;
}

__device__ __forceinline__ uint4 neg_bf(uint4 u) {
  return make_uint4(u.x ^ 0x80008000u, u.y ^ 0x80008000u, u.z ^ 0x80008000u, u.w ^ 0x80008000u);
}

// complex multiply-add straight into (re, im) accumulators:
// re += Re a Re x - Im a Im x (with a's Im planes negated), im += Re a Im x + Im a Re x
__device__ __forceinline__ void cstep2(const BfGroup& a, const BfGroup3& x, f16v& re, f16v& im) {
  re = rprod(a.hr, a.lr, x.hr, x.mr, x.lr, re);
  re = rprod(neg_bf(a.hi), neg_bf(a.li), x.hi, x.mi, x.li, re);
  im = rprod(a.hr, a.lr, x.hi, x.mi, x.li, im);
  im = rprod(a.hi, a.li, x.hr, x.mr, x.lr, im);
}

constexpr int BF_MC = 64;    // rows of a work item: BF_RT 32-row tiles
constexpr int BF_RT = BF_MC / 32;
constexpr int FRAG = 256;    // uint4 per operator fragment: 4 planes x 64 lanes
constexpr int VFRAG = 384;   // uint4 per T' fragment: 6 planes x 64 lanes

// per block of the partition: where its operator fragments are
struct BfBlock {
  int64_t off;    // first fragment in the pool (units of FRAG uint4)
  int64_t toff;   // far block of a row cluster above BF_MC rows: first T' fragment (units of VFRAG), else -1
  int g0, G;      // first global column group, number of column groups
  int KS, mt;     // contraction steps over the column groups (ceil(G / 2)); 32-row tiles of the block
  int R, T;       // far: stacked columns and 32-column tiles of them; near: 0, 0
};

// a work item: rows [r0, r0 + rows) of a row cluster and all its blocks
struct BfItem {
  int b0, nb;     // blocks rowblk[b0 .. b0 + nb)
  int rb, m;      // the row cluster: first position, rows
  int r0, rows;   // the item's rows within it (r0 a multiple of BF_MC, rows <= BF_MC)
  int lev;        // depth of the row cluster: its level buffer
  int pad;
};

// Every operand is stored in the order the matrix cores take it: a fragment
// holds one 32 x 16 operand tile as [plane][lane] 16-byte words, lane l = row
// l % 32 with the 8 values of contraction half l / 32, so that a wave reads a
// plane with one contiguous 1 KB load.
//   far block:  Vg[t][j]: rows c = 32 t + l % 32 of conj(Vbar)^T, column group
//               2 j + l / 32 of the block (zero beyond R or G);
//               Ug[rt][t][s]: rows i = 32 rt + l % 32 of Ubar, the eight
//               c = 32 t + 16 s + 8 (e / 4) + 4 h + e % 4 (h = l / 32), the order in
//               which an accumulator tile of T' (element r of lane half h holds
//               row 8 (r / 4) + 4 h + r % 4) feeds the next product (contraction
//               step s takes elements 8 s .. 8 s + 7)
//   near block: Dg[d][rt][j]: rows i = 32 rt + l % 32 of D_d, column group 2 j + l / 32
// Column groups are aligned to global cluster positions (group g covers
// positions 8 g .. 8 g + 7), like the right-hand side's.
__global__ void __launch_bounds__(256) bf_convert(const int* __restrict__ blk, const int* __restrict__ bterm,
                                                  const int64_t* __restrict__ toff,
                                                  const int64_t* __restrict__ cols, const int* __restrict__ bcol,
                                                  const cpx<float>* __restrict__ pool,
                                                  const BfBlock* __restrict__ bb, int nb,
                                                  uint4* __restrict__ out) {
  for (int b = blockIdx.x; b < nb; b += gridDim.x) {
    const BfBlock B = bb[b];
    if (B.G == 0) continue;
    const int rb = blk[5 * b], m = blk[5 * b + 1] - rb, cb = blk[5 * b + 2], n = blk[5 * b + 3] - cb;
    const bool adm = blk[5 * b + 4] & 1;
    uint4* base = out + B.off * FRAG;
    auto put = [&](int64_t frag, int l, const cpx<float>* v) {
      const BfGroup g = make_group(v);
      uint4* f = base + frag * FRAG + l;
      f[0] = g.hr;
      f[64] = g.lr;
      f[128] = g.hi;
      f[192] = g.li;
    };
    if (adm) {
      const cpx<float>* U = pool + cols[3 * bcol[b]];
      const cpx<float>* V = pool + cols[3 * bcol[b] + 1];
      const int nv = B.T * B.KS;
      for (int e = threadIdx.x; e < nv * 64; e += blockDim.x) {
        const int fr = e >> 6, l = e & 63, t = fr / B.KS, j = fr % B.KS;
        const int c = 32 * t + (l & 31), g = 2 * j + (l >> 5);
        cpx<float> v[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          const int jj = 8 * (B.g0 + g) + q - cb;
          const cpx<float> x =
              (c < B.R && g < B.G && jj >= 0 && jj < n) ? V[int64_t(c) * n + jj] : cpx<float>{0.f, 0.f};
          v[q] = {x.re, -x.im};   // conj(Vbar)
        }
        put(fr, l, v);
      }
      for (int e = threadIdx.x; e < B.mt * B.T * 2 * 64; e += blockDim.x) {
        const int fr = e >> 6, l = e & 63;
        const int rt = fr / (B.T * 2), t = (fr >> 1) % B.T, sd = fr & 1, h = l >> 5;
        const int i = 32 * rt + (l & 31);
        cpx<float> v[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          const int c = 32 * t + 16 * sd + 8 * (q >> 2) + 4 * h + (q & 3);
          v[q] = (i < m && c < B.R) ? U[int64_t(c) * m + i] : cpx<float>{0.f, 0.f};
        }
        put(int64_t(nv) + fr, l, v);
      }
    } else {
      const int nd = bterm[b + 1] - bterm[b];
      for (int e = threadIdx.x; e < nd * B.mt * B.KS * 64; e += blockDim.x) {
        const int fr = e >> 6, l = e & 63;
        const int d = fr / (B.mt * B.KS), rt = (fr / B.KS) % B.mt, j = fr % B.KS;
        const int i = 32 * rt + (l & 31), g = 2 * j + (l >> 5);
        const cpx<float>* D = pool + toff[bterm[b] + d];
        cpx<float> v[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          const int jj = 8 * (B.g0 + g) + q - cb;
          v[q] = (i < m && g < B.G && jj >= 0 && jj < n) ? D[int64_t(jj) * m + i] : cpx<float>{0.f, 0.f};
        }
        put(fr, l, v);
      }
    }
  }
}

// right-hand side in the operand order: Xg[kt][g][plane][32 lanes], lane = column
// kt * 32 + lane, the 8 values of positions 8 g .. 8 g + 7 (cluster order
// through perm, conjugated for conjugate-represented columns, zero beyond n)
__global__ void __launch_bounds__(256) bf_x_in(const cpx<float>* __restrict__ X, uint4* __restrict__ Xg,
                                               const int* __restrict__ perm, const int* __restrict__ conjflag,
                                               int n, int L, int ng, int nkt, int* __restrict__ counter) {
  if (blockIdx.x == 0 && threadIdx.x < 2) counter[threadIdx.x] = 0;   // work counter of the product
  const int64_t total = int64_t(nkt) * ng * 32;
  for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < total;
       e += int64_t(gridDim.x) * blockDim.x) {
    const int l = int(e & 31);
    const int64_t kg = e >> 5;
    const int kt = int(kg / ng), g = int(kg % ng);
    const int k = kt * 32 + l;
    cpx<float> v[8];
    const bool kin = k < L;
    const bool cj = kin && conjflag[k] != 0;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int p = 8 * g + q;
      const cpx<float> x = (kin && p < n) ? X[int64_t(k) * n + perm[p]] : cpx<float>{0.f, 0.f};
      v[q] = {x.re, cj ? -x.im : x.im};
    }
    const BfGroup3 G3 = make_group3(v);
    uint4* f = Xg + kg * 192 + l;
    f[0] = G3.hr;
    f[32] = G3.mr;
    f[64] = G3.lr;
    f[96] = G3.hi;
    f[128] = G3.mi;
    f[160] = G3.li;
  }
}

__device__ __forceinline__ BfGroup load_op(const uint4* __restrict__ f, int lane) {
  BfGroup g;
  g.hr = f[lane];
  g.lr = f[64 + lane];
  g.hi = f[128 + lane];
  g.li = f[192 + lane];
  return g;
}
// the lane's right-hand side group g (column tile base xk = Xg + kt * ng * 192)
__device__ __forceinline__ BfGroup3 load_x(const uint4* __restrict__ xk, int g, int lr) {
  const uint4* f = xk + int64_t(g) * 192 + lr;
  BfGroup3 x;
  x.hr = f[0];
  x.mr = f[32];
  x.lr = f[64];
  x.hi = f[96];
  x.mi = f[128];
  x.li = f[160];
  return x;
}



// T tile (stacked columns 32 t .. + 32 of a far block x the wave's 32
// frequency columns) = Vbar^H X_J, contracted over the block's column groups
__device__ __forceinline__ void t_tile(const uint4* __restrict__ Vg, const BfBlock& B, int t,
                                       const uint4* __restrict__ xk, int lane, int lr, int lh,
                                       f16v& re, f16v& im) {
  re = f16_zero();
  im = f16_zero();
  const uint4* vf = Vg + int64_t(t) * B.KS * FRAG;
  for (int j = 0; j < B.KS; ++j) {
    const int g = 2 * j + lh;
    const BfGroup a = load_op(vf + int64_t(j) * FRAG, lane);
    const BfGroup3 x = g < B.G ? load_x(xk, B.g0 + g, lr) : zero_group3();
    cstep2(a, x, re, im);
  }
}

// fiber of stacked column c of block b at frequency position kp
__device__ __forceinline__ cpx<float> fiber(const int64_t* __restrict__ cols, const cpx<float>* __restrict__ pool,
                                            int col0, int c, int kp) {
  return pool[cols[3 * (col0 + c) + 2] + kp];
}

// T' = F o T of the lane's 16 elements (rows 32 t + 8 (r / 4) + 4 h + r % 4, the lane's
// column), as two vector groups (contraction steps s = 0, 1)
__device__ __forceinline__ void t_prime(const f16v& re, const f16v& im, const BfBlock& B, int t, int col0,
                                        const int64_t* __restrict__ cols, const cpx<float>* __restrict__ pool,
                                        bool kin, int kp, int lh, BfGroup3& t0, BfGroup3& t1) {
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    cpx<float> v[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int r = 8 * s + e;
      const int c = 32 * t + 8 * (r >> 2) + 4 * lh + (r & 3);
      v[e] = {0.f, 0.f};
      if (c < B.R && kin) {
        const cpx<float> f = fiber(cols, pool, col0, c, kp);
        v[e] = {f.re * re[r] - f.im * im[r], f.re * im[r] + f.im * re[r]};
      }
    }
    (s == 0 ? t0 : t1) = make_group3(v);
  }
}

// T' of far blocks whose row cluster has more than BF_MC rows, into the T'
// buffer ([t][kt][s][plane][lane]); one workgroup per block, waves over
// (32-column tile, frequency tile) pairs
__global__ void __launch_bounds__(256) bf_tfill(const int* __restrict__ big, int nbig, const BfBlock* __restrict__ bb,
                                                const uint4* __restrict__ bfp, const int* __restrict__ bcol,
                                                const int64_t* __restrict__ cols, const cpx<float>* __restrict__ pool,
                                                const int* __restrict__ colpos, int L, int ng,
                                                const uint4* __restrict__ Xg, uint4* __restrict__ Tbuf) {
  const int lane = threadIdx.x & 63, lr = lane & 31, lh = lane >> 5;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), nw = blockDim.x >> 6;
  const int nkt = (L + 31) >> 5;
  for (int q = blockIdx.x; q < nbig; q += gridDim.x) {
    const int b = big[q];
    const BfBlock B = bb[b];
    const uint4* Vg = bfp + B.off * FRAG;
    for (int pr = w; pr < B.T * nkt; pr += nw) {
      const int t = pr / nkt, kt = pr % nkt;
      const int kcol = kt * 32 + lr;
      const bool kin = kcol < L;
      const int kp = kin ? colpos[kcol] : 0;
      f16v re, im;
      t_tile(Vg, B, t, Xg + int64_t(kt) * ng * 192, lane, lr, lh, re, im);
      BfGroup3 t0, t1;
      t_prime(re, im, B, t, bcol[b], cols, pool, kin, kp, lh, t0, t1);
      uint4* f = Tbuf + (B.toff + int64_t(t * nkt + kt) * 2) * VFRAG + lane;
      f[0] = t0.hr;
      f[64] = t0.mr;
      f[128] = t0.lr;
      f[192] = t0.hi;
      f[256] = t0.mi;
      f[320] = t0.li;
      f += VFRAG;
      f[0] = t1.hr;
      f[64] = t1.mr;
      f[128] = t1.lr;
      f[192] = t1.hi;
      f[256] = t1.mi;
      f[320] = t1.li;
    }
  }
}

__device__ __forceinline__ BfGroup3 load_t(const uint4* __restrict__ f, int lane) {
  BfGroup3 x;
  x.hr = f[lane];
  x.mr = f[64 + lane];
  x.lr = f[128 + lane];
  x.hi = f[192 + lane];
  x.mi = f[256 + lane];
  x.li = f[320 + lane];
  return x;
}

// the product: work items (rows of a row cluster, all its blocks) fetched from a
// counter; each wave owns 32-column frequency tiles and accumulates the item's
// rows in registers; plain stores into the row cluster's level buffer
__global__ void __launch_bounds__(256) bf_rows(
    const BfItem* __restrict__ items, int nitems, const int* __restrict__ rowblk, const int* __restrict__ blk,
    const int* __restrict__ bterm, const int64_t* __restrict__ tfoff, const int64_t* __restrict__ cols,
    const int* __restrict__ bcol, const cpx<float>* __restrict__ pool, const BfBlock* __restrict__ bb,
    const uint4* __restrict__ bfp, const int* __restrict__ colpos, int L, int ng,
    const uint4* __restrict__ Xg, const uint4* __restrict__ Tbuf, cpx<float>* __restrict__ Ylev,
    int64_t lev_stride, int* __restrict__ counter) {
  __shared__ int cur;
  const int lane = threadIdx.x & 63, lr = lane & 31, lh = lane >> 5;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), nw = blockDim.x >> 6;
  const int nkt = (L + 31) >> 5;
  while (true) {
    __syncthreads();
    if (threadIdx.x == 0) cur = atomicAdd(counter, 1);
    __syncthreads();
    const int it = cur;
    if (it >= nitems) break;
    const BfItem I = items[it];
    const int nrt = (I.rows + 31) >> 5;
    const int rt0 = I.r0 >> 5;
    for (int kt = w; kt < nkt; kt += nw) {
      const int kcol = kt * 32 + lr;
      const bool kin = kcol < L;
      const int kp = kin ? colpos[kcol] : 0;
      const uint4* xk = Xg + int64_t(kt) * ng * 192;
      f16v yre[BF_RT], yim[BF_RT];
#pragma unroll
      for (int rt = 0; rt < BF_RT; ++rt) yre[rt] = yim[rt] = f16_zero();
      for (int bi = 0; bi < I.nb; ++bi) {
        const int b = rowblk[I.b0 + bi];
        const BfBlock B = bb[b];
        if (B.G == 0) continue;
        const uint4* op = bfp + B.off * FRAG;
        if (!(blk[5 * b + 4] & 1)) {
          // near block: Y += f_d o (D_d X_J) per term and row tile
          const int d0 = bterm[b], nd = bterm[b + 1] - d0;
#pragma unroll
          for (int rt = 0; rt < BF_RT; ++rt) {
            if (rt >= nrt) break;
            for (int d = 0; d < nd; ++d) {
              const uint4* df = op + (int64_t(d) * B.mt + rt0 + rt) * B.KS * FRAG;
              f16v re = f16_zero(), im = f16_zero();
              for (int j = 0; j < B.KS; ++j) {
                const int g = 2 * j + lh;
                const BfGroup a = load_op(df + int64_t(j) * FRAG, lane);
                const BfGroup3 x = g < B.G ? load_x(xk, B.g0 + g, lr) : zero_group3();
                cstep2(a, x, re, im);
              }
              const cpx<float> f = kin ? pool[tfoff[d0 + d] + kp] : cpx<float>{0.f, 0.f};
#pragma unroll
              for (int r = 0; r < 16; ++r) {
                yre[rt][r] += f.re * re[r] - f.im * im[r];
                yim[rt][r] += f.re * im[r] + f.im * re[r];
              }
            }
          }
          continue;
        }
        // far block: per 32 stacked columns, T' (computed here, or read from the
        // T' buffer), then Y += Ubar[rows, tile] T'
        const uint4* Ug = op + int64_t(B.T) * B.KS * FRAG;
        for (int t = 0; t < B.T; ++t) {
          BfGroup3 t0, t1;
          if (B.toff < 0) {
            f16v re, im;
            t_tile(op, B, t, xk, lane, lr, lh, re, im);
            t_prime(re, im, B, t, bcol[b], cols, pool, kin, kp, lh, t0, t1);
          } else {
            const uint4* f = Tbuf + (B.toff + int64_t(t * nkt + kt) * 2) * VFRAG;
            t0 = load_t(f, lane);
            t1 = load_t(f + VFRAG, lane);
          }
#pragma unroll
          for (int rt = 0; rt < BF_RT; ++rt) {
            if (rt >= nrt) break;
            const uint4* uf = Ug + ((int64_t(rt0 + rt) * B.T + t) * 2) * FRAG;
            cstep2(load_op(uf, lane), t0, yre[rt], yim[rt]);
            cstep2(load_op(uf + FRAG, lane), t1, yre[rt], yim[rt]);
          }
        }
      }
      if (kin) {
        cpx<float>* yl = Ylev + I.lev * lev_stride;
#pragma unroll
        for (int rt = 0; rt < BF_RT; ++rt) {
          if (rt >= nrt) break;
#pragma unroll
          for (int r = 0; r < 16; ++r) {
            const int row = 32 * rt + 8 * (r >> 2) + 4 * lh + (r & 3);
            if (row < I.rows) yl[int64_t(I.rb + I.r0 + row) * L + kcol] = {yre[rt][r], yim[rt][r]};
          }
        }
      }
    }
  }
}

// Y[k][perm[p]] = sum over the levels of row p's row clusters (conjugated for
// conjugate-represented columns)
__global__ void bf_reduce_out(const cpx<float>* __restrict__ Ylev, int64_t lev_stride,
                              const unsigned* __restrict__ mask, cpx<float>* __restrict__ Y,
                              const int* __restrict__ perm, const int* __restrict__ conjflag, int n, int L) {
  const int64_t total = int64_t(n) * L;
  for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < total;
       e += int64_t(gridDim.x) * blockDim.x) {
    const int p = int(e / L), k = int(e % L);
    unsigned msk = mask[p];
    float re = 0.f, im = 0.f;
    while (msk) {
      const int d = __builtin_ctz(msk);
      msk &= msk - 1;
      const cpx<float> v = Ylev[d * lev_stride + e];
      re += v.re;
      im += v.im;
    }
    Y[int64_t(k) * n + perm[p]] = {re, conjflag[k] ? -im : im};
  }
}

// the operator's bf16 copy, work items, level masks; once per operator
int bf16_setup(gcq_context* ctx) {
  Faces3D& F = ctx->F;
  if (F.bf_valid) return GCQ_OK;
  const int nb = int(ctx->blocks.size());
  const int n = ctx->n, L = ctx->L;
  const int nkt = (L + 31) / 32;
  std::vector<BfBlock> bb(nb);
  std::vector<int> big;
  int64_t off = 0, toff = 0;
  for (int b = 0; b < nb; ++b) {
    const Block& Bk = ctx->blocks[b];
    const Cluster& A = ctx->clusters[Bk.row];
    const Cluster& C = ctx->clusters[Bk.col];
    const int m = A.end - A.begin;
    BfBlock& x = bb[b];
    x.off = off;
    x.toff = -1;
    x.g0 = C.begin / 8;
    x.G = (C.end + 7) / 8 - x.g0;
    x.KS = (x.G + 1) / 2;
    x.mt = (m + 31) / 32;
    x.R = x.T = 0;
    if (F.brank[b] == 0) {
      x.G = 0;
      continue;
    }
    if (Bk.admissible) {
      int R = 0;
      for (int d = F.bterm[b]; d < F.bterm[b + 1]; ++d) R += F.trank[d];
      x.R = R;
      x.T = (R + 31) / 32;
      if (R == 0) {
        x.G = 0;
        continue;
      }
      off += int64_t(x.T) * x.KS + int64_t(x.mt) * x.T * 2;
      if (m > BF_MC) {
        x.toff = toff;
        toff += int64_t(x.T) * nkt * 2;
        big.push_back(b);
      }
    } else {
      off += int64_t(F.brank[b]) * x.mt * x.KS;
    }
  }
  // work items: per row cluster with blocks, chunks of BF_MC rows, cost-ordered
  std::vector<std::vector<int>> byrow(ctx->clusters.size());
  for (int b = 0; b < nb; ++b)
    if (bb[b].G > 0) byrow[ctx->blocks[b].row].push_back(b);
  std::vector<int> rowblk;
  std::vector<BfItem> items;
  std::vector<double> cost;
  std::vector<unsigned> mask(n, 0u);
  for (size_t c = 0; c < byrow.size(); ++c) {
    if (byrow[c].empty()) continue;
    const Cluster& A = ctx->clusters[c];
    if (A.depth > 31) return fail(GCQ_ERR_UNSUPPORTED, "cluster tree deeper than 31 levels");
    const int m = A.end - A.begin;
    for (int p = A.begin; p < A.end; ++p) mask[p] |= 1u << A.depth;
    const int b0 = int(rowblk.size());
    rowblk.insert(rowblk.end(), byrow[c].begin(), byrow[c].end());
    for (int r0 = 0; r0 < m; r0 += BF_MC) {
      BfItem it;
      it.b0 = b0;
      it.nb = int(byrow[c].size());
      it.rb = A.begin;
      it.m = m;
      it.r0 = r0;
      it.rows = std::min(BF_MC, m - r0);
      it.lev = A.depth;
      it.pad = 0;
      const int nrt = (it.rows + 31) / 32;
      double wk = 0;
      for (int b : byrow[c]) {
        const BfBlock& x = bb[b];
        if (ctx->blocks[b].admissible)
          wk += double(x.T) * (x.toff < 0 ? x.KS + 2 * nrt : 3 * nrt);
        else
          wk += double(F.brank[b]) * nrt * x.KS;
      }
      items.push_back(it);
      cost.push_back(wk);
    }
  }
  std::vector<int> ord(items.size());
  std::iota(ord.begin(), ord.end(), 0);
  std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) { return cost[a] > cost[b]; });
  std::vector<BfItem> sitems(items.size());
  for (size_t a = 0; a < ord.size(); ++a) sitems[a] = items[ord[a]];
  int nlev = 0;
  for (auto& C : ctx->clusters) nlev = std::max(nlev, C.depth + 1);
  GCQ_TRY(F.bfpool.ensure(size_t(off) * FRAG * sizeof(uint4) + 256));
  GCQ_TRY(F.bftbuf.ensure(size_t(toff) * VFRAG * sizeof(uint4) + 256));
  GCQ_TRY(upload(F.d_bfblk, bb, ctx->stream));
  GCQ_TRY(upload(F.d_bfitems, sitems, ctx->stream));
  GCQ_TRY(upload(F.d_bfrowblk, rowblk, ctx->stream));
  GCQ_TRY(upload(F.d_bfbig, big, ctx->stream));
  GCQ_TRY(upload(F.d_bfmask, mask, ctx->stream));
  hipLaunchKernelGGL(bf_convert, dim3(std::min(nb, 65536)), dim3(256), 0, ctx->stream, ctx->d_blk.as<int>(),
                     F.d_bterm.as<int>(), F.d_toff.as<int64_t>(), F.d_cols.as<int64_t>(), F.d_bcol.as<int>(),
                     F.slices.as<cpx<float>>(), F.d_bfblk.as<BfBlock>(), nb, F.bfpool.as<uint4>());
  GCQ_HIP(hipGetLastError());
  GCQ_HIP(hipStreamSynchronize(ctx->stream));
  F.bf_items = int(sitems.size());
  F.bf_big = int(big.size());
  F.bf_levels = nlev;
  F.bf_bytes = off * FRAG * int64_t(sizeof(uint4));
  F.bf_valid = true;
  return GCQ_OK;
}

// the buffers of the product (in ctx->F.pxy): right-hand side fragments, work
// counter, level buffers
static size_t bf_xg_bytes(gcq_context* ctx) {
  const int ng = (ctx->n + 7) / 8, nkt = (ctx->L + 31) / 32;
  return size_t(nkt) * ng * 192 * sizeof(uint4);
}
size_t bf16_buffer_bytes(gcq_context* ctx) {
  return bf_xg_bytes(ctx) + 256 + size_t(ctx->F.bf_levels) * ctx->n * ctx->L * sizeof(cpx<float>) + 256;
}

// kernels of one product on stream st (no allocation, no host transfer)
void enqueue_perfreq_bf16(gcq_context* ctx, hipStream_t st, const void* X, void* Y) {
  Faces3D& F = ctx->F;
  const int n = ctx->n, L = ctx->L, ng = (n + 7) / 8, nkt = (L + 31) / 32;
  unsigned char* base = F.pxy.as<unsigned char>();
  uint4* Xg = reinterpret_cast<uint4*>(base);
  int* counter = reinterpret_cast<int*>(base + bf_xg_bytes(ctx));
  cpx<float>* Ylev = reinterpret_cast<cpx<float>*>(base + bf_xg_bytes(ctx) + 256);
  const int64_t lev_stride = int64_t(n) * L;
  const int* d_colpos = F.pmeta.as<int>();
  const int* d_conj = d_colpos + L;
  const int* perm = ctx->d_perm.as<int>();
  hipLaunchKernelGGL(bf_x_in, dim3(4096), dim3(256), 0, st, (const cpx<float>*)X, Xg, perm, d_conj, n, L, ng, nkt,
                     counter);
  if (F.bf_big > 0)
    hipLaunchKernelGGL(bf_tfill, dim3(std::min(F.bf_big, ctx->cus * 8)), dim3(256), 0, st, F.d_bfbig.as<int>(),
                       F.bf_big, F.d_bfblk.as<BfBlock>(), F.bfpool.as<uint4>(), F.d_bcol.as<int>(),
                       F.d_cols.as<int64_t>(), F.slices.as<cpx<float>>(), d_colpos, L, ng, (const uint4*)Xg,
                       F.bftbuf.as<uint4>());
  const int waves = std::min(4, nkt);
  hipLaunchKernelGGL(bf_rows, dim3(std::max(1, std::min(F.bf_items, ctx->cus * 8 / waves))), dim3(64 * waves), 0,
                     st, F.d_bfitems.as<BfItem>(), F.bf_items, F.d_bfrowblk.as<int>(), ctx->d_blk.as<int>(),
                     F.d_bterm.as<int>(), F.d_tfoff.as<int64_t>(), F.d_cols.as<int64_t>(), F.d_bcol.as<int>(),
                     F.slices.as<cpx<float>>(), F.d_bfblk.as<BfBlock>(), F.bfpool.as<uint4>(), d_colpos, L, ng,
                     (const uint4*)Xg, F.bftbuf.as<uint4>(), Ylev, lev_stride, counter);
  hipLaunchKernelGGL(bf_reduce_out, dim3(4096), dim3(256), 0, st, Ylev, lev_stride, F.d_bfmask.as<unsigned>(),
                     (cpx<float>*)Y, perm, d_conj, n, L);
}

}  // namespace gcq
