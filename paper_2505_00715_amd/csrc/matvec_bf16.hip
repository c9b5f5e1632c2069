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
// Operand storage: every operand in the order the matrix cores take it
// (fragments, below), 16-byte aligned loads of 8 bf16 values.  The product per
// frequency column, as in the float kernel -- far block: T = Vbar^H X_J
// (stacked columns x columns), T' = F o T (fibers), Y_I += Ubar T'; near block:
// Y_I += sum_d f_d o (D_d X_J).  Work items are rows of one row cluster with all
// its far (or all its near) blocks; a workgroup's waves own the frequency
// columns, accumulate the item's rows in registers and store them once into
// the level buffer of the cluster's depth (near blocks: the level after the
// deepest); a last pass sums the levels of each row into Y.  No atomics.
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
constexpr int BF_NX = 8;     // work lists of the product, one per XCD (workgroup i runs on XCD i % 8)
constexpr int BF_WAVES = 8;  // waves of a workgroup: one 32-column frequency tile each (256 columns)
constexpr int BF_RTB = 3;    // 32-row tiles of a work item on a row cluster above BF_MC rows (T' from the buffer)
constexpr int BF_COUNTERS = 4 * BF_NX;   // work counters: lists of far items (small, big row clusters), near items, T' blocks
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
  if (blockIdx.x == 0 && threadIdx.x < BF_COUNTERS) counter[threadIdx.x] = 0;   // work counters of the product
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



// some of the tiles kt0 .. kt0 + KW - 1 is to be computed (no mask: all are)
template <int KW>
__device__ __forceinline__ bool tiles_active(const int* __restrict__ tmask, int kt0, int nkt) {
  if (!tmask) return true;
  bool any = false;
#pragma unroll
  for (int u = 0; u < KW; ++u) any = any || (kt0 + u < nkt && tmask[kt0 + u] != 0);
  return any;
}

// the KW 32-column frequency tiles kt0 .. kt0 + KW - 1 that a wave owns
template <int KW>
struct Tiles {
  int kcol[KW];            // the lane's column in each tile
  bool kin[KW];            // that column exists (kcol < L)
  bool kv[KW];             // the tile exists (kt < number of tiles)
  int kp[KW];              // frequency position of the lane's column
  const uint4* xk[KW];     // the tile's right-hand side fragments
  __device__ __forceinline__ Tiles(int kt0, int nkt, int L, int lr, int ng, const int* __restrict__ colpos,
                                   const uint4* __restrict__ Xg) {
#pragma unroll
    for (int u = 0; u < KW; ++u) {
      const int kt = kt0 + u;
      kv[u] = kt < nkt;
      kcol[u] = kt * 32 + lr;
      kin[u] = kv[u] && kcol[u] < L;
      kp[u] = kin[u] ? colpos[kcol[u]] : 0;
      xk[u] = Xg + int64_t(kv[u] ? kt : 0) * ng * 192;
    }
  }
};

// T tile (stacked columns 32 t .. + 32 of a far block x 32 frequency columns)
// = Vbar^H X_J for each of the wave's tiles, contracted over the block's column
// groups; each Vbar fragment serves all KW tiles
template <int KW>
__device__ __forceinline__ void t_tile(const uint4* __restrict__ Vg, const BfBlock& B, int t, const Tiles<KW>& C,
                                       int lane, int lr, int lh, f16v* re, f16v* im) {
#pragma unroll
  for (int u = 0; u < KW; ++u) re[u] = im[u] = f16_zero();
  const uint4* vf = Vg + int64_t(t) * B.KS * FRAG;
  for (int j = 0; j < B.KS; ++j) {
    const int g = 2 * j + lh;
    const BfGroup a = load_op(vf + int64_t(j) * FRAG, lane);
#pragma unroll
    for (int u = 0; u < KW; ++u) {
      const BfGroup3 x = (g < B.G && C.kv[u]) ? load_x(C.xk[u], B.g0 + g, lr) : zero_group3();
      cstep2(a, x, re[u], im[u]);
    }
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

// next work item of a workgroup: from its XCD's list (spatially ordered, so
// that the row clusters in flight on one XCD share their blocks' column vectors
// in its L2), then from the other lists; -1 when all are done.  range holds
// BF_NX + 1 list bounds, counter BF_NX counters.
__device__ __forceinline__ int next_item(const int* __restrict__ range, int* __restrict__ counter, int home,
                                         int& visited, int* cur) {
  __syncthreads();
  if (threadIdx.x == 0) {
    int got = -1;
    while (visited < BF_NX) {
      const int li = (home + visited) % BF_NX;
      const int q = atomicAdd(counter + li, 1);
      if (q < range[li + 1] - range[li]) {
        got = range[li] + q;
        break;
      }
      ++visited;
    }
    *cur = got;
  }
  __syncthreads();
  // wave-uniform: the item's and its blocks' descriptors then live in scalar registers
  return __builtin_amdgcn_readfirstlane(*cur);
}

__device__ __forceinline__ void store_t(uint4* __restrict__ f, const BfGroup3& a) {
  f[0] = a.hr;
  f[64] = a.mr;
  f[128] = a.lr;
  f[192] = a.hi;
  f[256] = a.mi;
  f[320] = a.li;
}

// T' of far blocks whose row cluster has more than BF_MC rows, into the T'
// buffer ([t][kt][s][plane][lane]); one workgroup per block, blocks from the
// workgroup's XCD list (ordered by column cluster, so that blocks in flight on
// an XCD share their right-hand side in its L2), each wave KW
// 32-column frequency tiles, the stacked columns in groups of BF_TG tiles, so
// that each right-hand side fragment serves BF_TG tiles and each Vbar fragment
// KW tiles
constexpr int BF_TG = 2;
template <int KW>
__global__ void __launch_bounds__(KW == 1 ? 512 : 256, KW == 1 ? 4 : 1) bf_tfill(
    const int* __restrict__ big, const int* __restrict__ range, int* __restrict__ counter,
    const BfBlock* __restrict__ bb, const uint4* __restrict__ bfp,
    const int* __restrict__ bcol, const int64_t* __restrict__ cols, const cpx<float>* __restrict__ pool,
    const int* __restrict__ colpos, int L, int ng, const uint4* __restrict__ Xg, uint4* __restrict__ Tbuf,
    const int* __restrict__ tmask) {
  const int lane = threadIdx.x & 63, lr = lane & 31, lh = lane >> 5;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), nw = blockDim.x >> 6;
  const int nkt = (L + 31) >> 5;
  __shared__ int cur;
  int visited = 0;
  for (int q; (q = next_item(range, counter, blockIdx.x % BF_NX, visited, &cur)) >= 0;) {
    const int b = big[q];
    const BfBlock B = bb[b];
    const uint4* Vg = bfp + B.off * FRAG;
    for (int kt0 = w * KW; kt0 < nkt; kt0 += nw * KW) {
      if (!tiles_active<KW>(tmask, kt0, nkt)) continue;
      const Tiles<KW> C(kt0, nkt, L, lr, ng, colpos, Xg);
      for (int t0 = 0; t0 < B.T; t0 += BF_TG) {
        const int nt = min(BF_TG, B.T - t0);
        f16v re[BF_TG][KW], im[BF_TG][KW];
#pragma unroll
        for (int v = 0; v < BF_TG; ++v)
#pragma unroll
          for (int u = 0; u < KW; ++u) re[v][u] = im[v][u] = f16_zero();
        for (int j = 0; j < B.KS; ++j) {
          const int g = 2 * j + lh;
          BfGroup3 x[KW];
#pragma unroll
          for (int u = 0; u < KW; ++u) x[u] = (g < B.G && C.kv[u]) ? load_x(C.xk[u], B.g0 + g, lr) : zero_group3();
#pragma unroll
          for (int v = 0; v < BF_TG; ++v) {
            if (v >= nt) break;
            const BfGroup a = load_op(Vg + (int64_t(t0 + v) * B.KS + j) * FRAG, lane);
#pragma unroll
            for (int u = 0; u < KW; ++u) cstep2(a, x[u], re[v][u], im[v][u]);
          }
        }
#pragma unroll
        for (int v = 0; v < BF_TG; ++v) {
          if (v >= nt) break;
          const int t = t0 + v;
#pragma unroll
          for (int u = 0; u < KW; ++u) {
            if (!C.kv[u]) continue;
            BfGroup3 a, c;
            t_prime(re[v][u], im[v][u], B, t, bcol[b], cols, pool, C.kin[u], C.kp[u], lh, a, c);
            uint4* f = Tbuf + (B.toff + int64_t(t * nkt + kt0 + u) * 2) * VFRAG + lane;
            store_t(f, a);
            store_t(f + VFRAG, c);
          }
        }
      }
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

// stores of a wave's accumulated rows (its 32-column tile) into a level buffer
template <int RT>
__device__ __forceinline__ void store_rows(const f16v* yre, const f16v* yim, int nrt, const BfItem& I, int lh,
                                           int kcol, int L, cpx<float>* __restrict__ yl) {
#pragma unroll
  for (int rt = 0; rt < RT; ++rt) {
    if (rt >= nrt) break;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int row = 32 * rt + 8 * (r >> 2) + 4 * lh + (r & 3);
      if (row < I.rows) yl[int64_t(I.rb + I.r0 + row) * L + kcol] = {yre[rt][r], yim[rt][r]};
    }
  }
}

// far blocks of the product: work items (rows of a row cluster, all its far
// blocks); each wave owns KW 32-column frequency tiles (all L columns in one
// pass, so the workgroup fetches each operator fragment once, and each
// fragment a wave loads serves KW tiles) and accumulates the item's rows in
// registers; per 32 stacked columns of a block, T' (BIG: read from the T'
// buffer, items of up to 32 BF_RTB rows; else computed here, items of up to
// BF_MC rows), then Y += Ubar[rows, tile] T'; plain stores into the row
// cluster's level buffer
template <bool BIG, int KW>
__global__ void __launch_bounds__(KW == 1 ? 512 : 256) bf_rows(
    const BfItem* __restrict__ items, const int* __restrict__ range, const int* __restrict__ rowblk,
    const int64_t* __restrict__ cols, const int* __restrict__ bcol, const cpx<float>* __restrict__ pool,
    const BfBlock* __restrict__ bb, const uint4* __restrict__ bfp, const int* __restrict__ colpos, int L, int ng,
    const uint4* __restrict__ Xg, const uint4* __restrict__ Tbuf, cpx<float>* __restrict__ Ylev,
    int64_t lev_stride, int* __restrict__ counter, const int* __restrict__ tmask) {
  constexpr int RT = BIG ? BF_RTB : BF_RT;
  __shared__ int cur;
  const int lane = threadIdx.x & 63, lr = lane & 31, lh = lane >> 5;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), nw = blockDim.x >> 6;
  const int nkt = (L + 31) >> 5;
  int visited = 0;
  for (int it; (it = next_item(range, counter, blockIdx.x % BF_NX, visited, &cur)) >= 0;) {
    const BfItem I = items[it];
    const int nrt = (I.rows + 31) >> 5;
    const int rt0 = I.r0 >> 5;
    for (int kt0 = w * KW; kt0 < nkt; kt0 += nw * KW) {
      if (!tiles_active<KW>(tmask, kt0, nkt)) continue;
      const Tiles<KW> C(kt0, nkt, L, lr, ng, colpos, Xg);
      f16v yre[KW][RT], yim[KW][RT];
#pragma unroll
      for (int u = 0; u < KW; ++u)
#pragma unroll
        for (int rt = 0; rt < RT; ++rt) yre[u][rt] = yim[u][rt] = f16_zero();
      for (int bi = 0; bi < I.nb; ++bi) {
        const int b = rowblk[I.b0 + bi];
        const BfBlock B = bb[b];
        const uint4* op = bfp + B.off * FRAG;
        const uint4* Ug = op + int64_t(B.T) * B.KS * FRAG;
        if constexpr (BIG) {
          // the block's T' halves (t, sd) in order, the next one loaded while
          // the current one is applied; one row tile's fragments in flight (the
          // compiler barriers keep the loads of all row tiles from being
          // hoisted together, which would not fit the registers)
          auto tload = [&](int h, BfGroup3* tv) {
#pragma unroll
            for (int u = 0; u < KW; ++u)
              tv[u] = C.kv[u] ? load_t(Tbuf + (B.toff + int64_t((h >> 1) * nkt + kt0 + u) * 2 + (h & 1)) * VFRAG,
                                       lane)
                              : zero_group3();
          };
          BfGroup3 nxt[KW];
          tload(0, nxt);
          for (int h = 0; h < 2 * B.T; ++h) {
            BfGroup3 tv[KW];
#pragma unroll
            for (int u = 0; u < KW; ++u) tv[u] = nxt[u];
            if (h + 1 < 2 * B.T) tload(h + 1, nxt);
            const int t = h >> 1, sd = h & 1;
#pragma unroll
            for (int rt = 0; rt < RT; ++rt) {
              if (rt >= nrt) break;
              const BfGroup a = load_op(Ug + ((int64_t(rt0 + rt) * B.T + t) * 2 + sd) * FRAG, lane);
#pragma unroll
              for (int u = 0; u < KW; ++u) cstep2(a, tv[u], yre[u][rt], yim[u][rt]);
              asm volatile("" ::: "memory");
            }
          }
          continue;
        }
        for (int t = 0; t < B.T; ++t) {
          {
            f16v re[KW], im[KW];
            t_tile<KW>(op, B, t, C, lane, lr, lh, re, im);
            BfGroup3 t0[KW], t1[KW];
#pragma unroll
            for (int u = 0; u < KW; ++u)
              t_prime(re[u], im[u], B, t, bcol[b], cols, pool, C.kin[u], C.kp[u], lh, t0[u], t1[u]);
#pragma unroll
            for (int rt = 0; rt < RT; ++rt) {
              if (rt >= nrt) break;
              const uint4* uf = Ug + ((int64_t(rt0 + rt) * B.T + t) * 2) * FRAG;
              const BfGroup a0 = load_op(uf, lane);
#pragma unroll
              for (int u = 0; u < KW; ++u) cstep2(a0, t0[u], yre[u][rt], yim[u][rt]);
              const BfGroup a1 = load_op(uf + FRAG, lane);
#pragma unroll
              for (int u = 0; u < KW; ++u) cstep2(a1, t1[u], yre[u][rt], yim[u][rt]);
            }
          }
        }
      }
#pragma unroll
      for (int u = 0; u < KW; ++u)
        if (C.kin[u]) store_rows<RT>(yre[u], yim[u], nrt, I, lh, C.kcol[u], L, Ylev + I.lev * lev_stride);
    }
  }
}

// near blocks of the product: work items (rows of a row cluster, all its
// inadmissible blocks); each wave owns one 32-row tile and one 32-column
// frequency tile (BF_WAVES x BF_RT waves: registers for one row tile only, so
// four waves fit a SIMD); Y += f_d o (D_d X_J) per term; plain stores into the
// near-field buffer (the level after the tree's deepest)
__global__ void __launch_bounds__(BF_WAVES * BF_RT * 64) bf_near(
    const BfItem* __restrict__ items, const int* __restrict__ range, const int* __restrict__ rowblk,
    const int* __restrict__ bterm, const int64_t* __restrict__ tfoff, const cpx<float>* __restrict__ pool,
    const BfBlock* __restrict__ bb, const uint4* __restrict__ bfp, const int* __restrict__ colpos, int L, int ng,
    const uint4* __restrict__ Xg, cpx<float>* __restrict__ Ylev, int64_t lev_stride, int* __restrict__ counter,
    int wk, const int* __restrict__ tmask) {
  __shared__ int cur;
  const int lane = threadIdx.x & 63, lr = lane & 31, lh = lane >> 5;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int wrt = w / wk, wkt = w % wk;   // the wave's row tile and first frequency tile
  const int nkt = (L + 31) >> 5;
  int visited = 0;
  for (int it; (it = next_item(range, counter, blockIdx.x % BF_NX, visited, &cur)) >= 0;) {
    const BfItem I = items[it];
    const int nrt = (I.rows + 31) >> 5;
    if (wrt >= nrt) continue;   // (next_item's barriers are reached by every wave)
    const int rt = (I.r0 >> 5) + wrt;
    for (int kt = wkt; kt < nkt; kt += wk) {
      if (tmask && !tmask[kt]) continue;
      const Tiles<1> C(kt, nkt, L, lr, ng, colpos, Xg);
      f16v yre = f16_zero(), yim = f16_zero();
      for (int bi = 0; bi < I.nb; ++bi) {
        const int b = rowblk[I.b0 + bi];
        const BfBlock B = bb[b];
        const uint4* op = bfp + B.off * FRAG;
        const int d0 = bterm[b], nd = bterm[b + 1] - d0;
        for (int d = 0; d < nd; ++d) {
          f16v tre = f16_zero(), tim = f16_zero();
          const uint4* df = op + (int64_t(d) * B.mt + rt) * B.KS * FRAG;
          for (int j = 0; j < B.KS; ++j) {
            const int g = 2 * j + lh;
            const BfGroup3 x = (g < B.G && C.kv[0]) ? load_x(C.xk[0], B.g0 + g, lr) : zero_group3();
            cstep2(load_op(df + int64_t(j) * FRAG, lane), x, tre, tim);
          }
          const cpx<float> f = C.kin[0] ? pool[tfoff[d0 + d] + C.kp[0]] : cpx<float>{0.f, 0.f};
#pragma unroll
          for (int r = 0; r < 16; ++r) {
            yre[r] += f.re * tre[r] - f.im * tim[r];
            yim[r] += f.re * tim[r] + f.im * tre[r];
          }
        }
      }
      if (C.kin[0]) {
        cpx<float>* yl = Ylev + I.lev * lev_stride;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int row = 32 * wrt + 8 * (r >> 2) + 4 * lh + (r & 3);
          if (row < I.rows) yl[int64_t(I.rb + I.r0 + row) * L + C.kcol[0]] = {yre[r], yim[r]};
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
  // work items: per row cluster, chunks of BF_MC rows with all its far blocks
  // (far items, stored into the level of the cluster's depth) and with all its
  // near blocks (near items, stored into the level after the deepest)
  int nlev = 0;
  for (auto& C : ctx->clusters) nlev = std::max(nlev, C.depth + 1);
  if (nlev > 31) return fail(GCQ_ERR_UNSUPPORTED, "cluster tree deeper than 31 levels");
  // kinds: 0 far blocks of row clusters up to BF_MC rows (T' computed in the
  // item), 1 far blocks of larger row clusters (T' from the buffer), 2 near blocks
  std::vector<std::vector<int>> byrow[3];
  for (auto& v : byrow) v.resize(ctx->clusters.size());
  for (int b = 0; b < nb; ++b) {
    if (bb[b].G == 0) continue;
    const int r = ctx->blocks[b].row;
    const int kind = ctx->blocks[b].admissible ? (bb[b].toff >= 0 ? 1 : 0) : 2;
    byrow[kind][r].push_back(b);
  }
  std::vector<int> rowblk;
  std::vector<BfItem> sitems;
  std::vector<int> range;   // BF_NX + 1 bounds of the lists of each kind
  std::vector<unsigned> mask(n, 0u);
  for (int kind = 0; kind < 3; ++kind) {
    std::vector<BfItem> items;
    std::vector<double> cost;
    const int chunk = kind == 1 ? 32 * BF_RTB : BF_MC;
    for (size_t c = 0; c < byrow[kind].size(); ++c) {
      const std::vector<int>& bl = byrow[kind][c];
      if (bl.empty()) continue;
      const Cluster& A = ctx->clusters[c];
      const int m = A.end - A.begin;
      const int lev = kind < 2 ? A.depth : nlev;
      for (int p = A.begin; p < A.end; ++p) mask[p] |= 1u << lev;
      const int b0 = int(rowblk.size());
      rowblk.insert(rowblk.end(), bl.begin(), bl.end());
      for (int r0 = 0; r0 < m; r0 += chunk) {
        BfItem it;
        it.b0 = b0;
        it.nb = int(bl.size());
        it.rb = A.begin;
        it.m = m;
        it.r0 = r0;
        it.rows = std::min(chunk, m - r0);
        it.lev = lev;
        it.pad = 0;
        const int nrt = (it.rows + 31) / 32;
        double wk = 0;
        for (int b : bl) {
          const BfBlock& x = bb[b];
          if (kind == 0)
            wk += double(x.T) * (x.KS + 2 * nrt);
          else if (kind == 1)
            wk += double(x.T) * 3 * nrt;
          else
            wk += double(F.brank[b]) * nrt * x.KS;
        }
        items.push_back(it);
        cost.push_back(wk);
      }
    }
    // spatial order (first row), cut into BF_NX consecutive lists of equal cost
    std::vector<int> ord(items.size());
    std::iota(ord.begin(), ord.end(), 0);
    std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) {
      return items[a].rb + items[a].r0 < items[b].rb + items[b].r0;
    });
    const int base = int(sitems.size());
    for (int a : ord) sitems.push_back(items[a]);
    std::vector<int> r(BF_NX + 1, int(sitems.size()));
    r[0] = base;
    double total = 0, acc = 0;
    for (double c : cost) total += c;
    int x = 1;
    for (size_t a = 0; a < ord.size() && x < BF_NX; ++a) {
      acc += cost[ord[a]];
      while (x < BF_NX && acc >= total * x / BF_NX) r[x++] = base + int(a + 1);
    }
    range.insert(range.end(), r.begin(), r.end());
  }
  // T' blocks: ordered by column cluster, cut into BF_NX lists of equal work
  std::stable_sort(big.begin(), big.end(), [&](int a, int b) {
    return bb[a].g0 != bb[b].g0 ? bb[a].g0 < bb[b].g0 : a < b;
  });
  {
    double total = 0, acc = 0;
    for (int b : big) total += double(bb[b].T) * bb[b].KS;
    std::vector<int> r(BF_NX + 1, int(big.size()));
    r[0] = 0;
    int x = 1;
    for (size_t a = 0; a < big.size() && x < BF_NX; ++a) {
      acc += double(bb[big[a]].T) * bb[big[a]].KS;
      while (x < BF_NX && acc >= total * x / BF_NX) r[x++] = int(a + 1);
    }
    range.insert(range.end(), r.begin(), r.end());
  }
  GCQ_TRY(F.bfpool.ensure(size_t(off) * FRAG * sizeof(uint4) + 256));
  GCQ_TRY(F.bftbuf.ensure(size_t(toff) * VFRAG * sizeof(uint4) + 256));
  GCQ_TRY(upload(F.d_bfblk, bb, ctx->stream));
  GCQ_TRY(upload(F.d_bfitems, sitems, ctx->stream));
  GCQ_TRY(upload(F.d_bfrange, range, ctx->stream));
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
  F.bf_levels = nlev + 1;
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

// the T' fill and the row kernels with KW 32-column tiles per wave
template <int KW>
static void enqueue_bf_kernels(gcq_context* ctx, hipStream_t st, const uint4* Xg, int* counter, cpx<float>* Ylev,
                               int64_t lev_stride, const int* d_colpos, const int* tmask) {
  Faces3D& F = ctx->F;
  const int n = ctx->n, L = ctx->L, ng = (n + 7) / 8, nkt = (L + 31) / 32;
  const int waves = std::max(1, std::min(BF_WAVES / KW, (nkt + KW - 1) / KW));
  const int* range = F.d_bfrange.as<int>();
  if (F.bf_big > 0)
    hipLaunchKernelGGL(bf_tfill<KW>, dim3(ctx->cus * 2), dim3(64 * waves), 0, st, F.d_bfbig.as<int>(),
                       range + 3 * (BF_NX + 1), counter + 3 * BF_NX, F.d_bfblk.as<BfBlock>(), F.bfpool.as<uint4>(),
                       F.d_bcol.as<int>(), F.d_cols.as<int64_t>(), F.slices.as<cpx<float>>(), d_colpos, L, ng, Xg,
                       F.bftbuf.as<uint4>(), tmask);
  hipLaunchKernelGGL((bf_rows<false, KW>), dim3(ctx->cus * 2), dim3(64 * waves), 0, st, F.d_bfitems.as<BfItem>(),
                     range, F.d_bfrowblk.as<int>(), F.d_cols.as<int64_t>(), F.d_bcol.as<int>(),
                     F.slices.as<cpx<float>>(), F.d_bfblk.as<BfBlock>(), F.bfpool.as<uint4>(), d_colpos, L, ng, Xg,
                     F.bftbuf.as<uint4>(), Ylev, lev_stride, counter, tmask);
  // row clusters above BF_MC rows: two tiles per wave in either case (measured
  // faster, and one tile per wave with the T' prefetch does not fit 256 registers;
  // one row tile per wave on 64-row items reads the T' buffer more: slower)
  const int bwaves = std::max(1, std::min(BF_WAVES / 2, (nkt + 1) / 2));
  hipLaunchKernelGGL((bf_rows<true, 2>), dim3(ctx->cus * 2), dim3(64 * bwaves), 0, st, F.d_bfitems.as<BfItem>(),
                     range + BF_NX + 1, F.d_bfrowblk.as<int>(), F.d_cols.as<int64_t>(), F.d_bcol.as<int>(),
                     F.slices.as<cpx<float>>(), F.d_bfblk.as<BfBlock>(), F.bfpool.as<uint4>(), d_colpos, L, ng,
                     Xg, F.bftbuf.as<uint4>(), Ylev, lev_stride, counter + BF_NX, tmask);
  // near blocks: one frequency tile and one row tile per wave
  const int nwk = std::min(BF_WAVES, nkt);
  hipLaunchKernelGGL(bf_near, dim3(ctx->cus * 2), dim3(64 * nwk * BF_RT), 0, st, F.d_bfitems.as<BfItem>(),
                     range + 2 * (BF_NX + 1), F.d_bfrowblk.as<int>(), F.d_bterm.as<int>(), F.d_tfoff.as<int64_t>(),
                     F.slices.as<cpx<float>>(), F.d_bfblk.as<BfBlock>(), F.bfpool.as<uint4>(), d_colpos, L, ng, Xg,
                     Ylev, lev_stride, counter + 2 * BF_NX, nwk, tmask);
}

// kernels of one product on stream st (no allocation, no host transfer)
void enqueue_perfreq_bf16(gcq_context* ctx, hipStream_t st, const void* X, void* Y, const int* tile_mask) {
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
  if (ctx->tune.product_cols_per_wave == 64)
    enqueue_bf_kernels<2>(ctx, st, Xg, counter, Ylev, lev_stride, d_colpos, tile_mask);
  else
    enqueue_bf_kernels<1>(ctx, st, Xg, counter, Ylev, lev_stride, d_colpos, tile_mask);
  hipLaunchKernelGGL(bf_reduce_out, dim3(4096), dim3(256), 0, st, Ylev, lev_stride, F.d_bfmask.as<unsigned>(),
                     (cpx<float>*)Y, perm, d_conj, n, L);
}

}  // namespace gcq
