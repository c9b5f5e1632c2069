// Device-side building blocks shared by the library's kernels: complex
// arithmetic, wave64 reductions, the panel table, and evaluation of the
// Laplace-domain single-layer entries V(s)[i, j] (three quadrature tiers).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gcq {

constexpr int WAVE = 64;
constexpr int NQ_FAR = 7;       // 7-point degree-5 rule
constexpr int NQ_NEAR = 112;    // 7 points on 16 sub-triangles
constexpr int NGL = 16;         // Gauss-Legendre points of the self panel

template <typename T>
struct cpx {
  T re, im;
};

template <typename T>
__device__ __forceinline__ cpx<T> cmul(cpx<T> a, cpx<T> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename T>
__device__ __forceinline__ cpx<T> cmulc(cpx<T> a, cpx<T> b) {  // conj(a) * b
  return {a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re};
}
template <typename T>
__device__ __forceinline__ T cabs2(cpx<T> a) {
  return a.re * a.re + a.im * a.im;
}
// squared modulus in double: pivot searches on float data must not lose
// entries whose square underflows in float
template <typename T>
__device__ __forceinline__ double mag2(cpx<T> a) {
  return double(a.re) * double(a.re) + double(a.im) * double(a.im);
}
// smallest squared modulus a pivot may have: its reciprocal must stay finite
template <typename T>
struct PivFloor;
template <>
struct PivFloor<float> {
  static constexpr double v = 1.4e-76;  // (FLT_MIN)^2
};
template <>
struct PivFloor<double> {
  static constexpr double v = 0.0;
};
template <typename T>
__device__ __forceinline__ cpx<T> cinv(cpx<T> a) {
  const double m = mag2(a);
  return {T(double(a.re) / m), T(-double(a.im) / m)};
}

// ---- wave64 reductions (every lane receives the result) --------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, WAVE);
  return v;
}
__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, WAVE);
  return v;
}
__device__ __forceinline__ int wave_min_int(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, WAVE));
  return v;
}
__device__ __forceinline__ int wave_max_int(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, WAVE));
  return v;
}
// argmax of (val, idx) pairs: largest val, lowest idx among equal vals.
// Lanes without a candidate pass val = -1.
template <typename T>
__device__ __forceinline__ void wave_argmax(T& val, int& idx) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    T ov = __shfl_xor(val, o, WAVE);
    int oi = __shfl_xor(idx, o, WAVE);
    if (ov > val || (ov == val && oi < idx)) {
      val = ov;
      idx = oi;
    }
  }
}

// ---- wave-uniform values ----------------------------------------------------
// A value that every lane holds alike (a group reduction's result, a value read
// from LDS by all lanes) is moved to a scalar register, which frees vector
// registers for the loops.
__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ int64_t uni64(int64_t v) {
  const int lo = __builtin_amdgcn_readfirstlane(int(uint32_t(uint64_t(v))));
  const int hi = __builtin_amdgcn_readfirstlane(int(uint32_t(uint64_t(v) >> 32)));
  return int64_t((uint64_t(uint32_t(hi)) << 32) | uint64_t(uint32_t(lo)));
}
__device__ __forceinline__ double unid(double v) {
  return __builtin_bit_cast(double, uni64(__builtin_bit_cast(int64_t, v)));
}

// ---- group reductions: NW wave64s of one workgroup -------------------------
// Every thread of the workgroup receives the result.  The waves' partial
// results are combined in wave order, so the result does not depend on timing.
// Each call starts with a barrier, which protects the exchange slots from the
// previous call's readers.
template <int NW>
__device__ __forceinline__ double grp_sum(double v) {
  v = wave_sum(v);
  if constexpr (NW > 1) {
    __shared__ double red[NW];
    __syncthreads();
    if ((threadIdx.x & (WAVE - 1)) == 0) red[threadIdx.x / WAVE] = v;
    __syncthreads();
    v = red[0];
#pragma unroll
    for (int w = 1; w < NW; ++w) v += red[w];
  }
  return v;
}
template <int NW>
__device__ __forceinline__ void grp_sum2(double& a, double& b) {
  a = wave_sum(a);
  b = wave_sum(b);
  if constexpr (NW > 1) {
    __shared__ double red[2 * NW];
    __syncthreads();
    if ((threadIdx.x & (WAVE - 1)) == 0) {
      red[2 * (threadIdx.x / WAVE)] = a;
      red[2 * (threadIdx.x / WAVE) + 1] = b;
    }
    __syncthreads();
    a = red[0];
    b = red[1];
#pragma unroll
    for (int w = 1; w < NW; ++w) {
      a += red[2 * w];
      b += red[2 * w + 1];
    }
  }
}
template <int NW>
__device__ __forceinline__ int grp_min_int(int v) {
  v = wave_min_int(v);
  if constexpr (NW > 1) {
    __shared__ int red[NW];
    __syncthreads();
    if ((threadIdx.x & (WAVE - 1)) == 0) red[threadIdx.x / WAVE] = v;
    __syncthreads();
    v = red[0];
#pragma unroll
    for (int w = 1; w < NW; ++w) v = min(v, red[w]);
  }
  return v;
}
// argmax over the group: largest val, lowest idx among equal vals
template <int NW>
__device__ __forceinline__ void grp_argmax(double& val, int& idx) {
  wave_argmax(val, idx);
  if constexpr (NW > 1) {
    __shared__ double rv[NW];
    __shared__ int ri[NW];
    __syncthreads();
    if ((threadIdx.x & (WAVE - 1)) == 0) {
      rv[threadIdx.x / WAVE] = val;
      ri[threadIdx.x / WAVE] = idx;
    }
    __syncthreads();
    val = rv[0];
    idx = ri[0];
#pragma unroll
    for (int w = 1; w < NW; ++w)
      if (rv[w] > val || (rv[w] == val && ri[w] < idx)) {
        val = rv[w];
        idx = ri[w];
      }
  }
}

// ---- constant tables (filled by the host at context creation) --------------
struct Consts {
  double gl_x[NGL], gl_w[NGL];        // Gauss-Legendre on [0, 1]
  double nb[NQ_NEAR][3];              // barycentric points of the near rule
  double nw[NQ_NEAR];                 // weights (sum 1) of the near rule
};

// ---- panel table (cluster-permuted order, structure of arrays) --------------
// q64/q32 hold 28 arrays of n: qx[7], qy[7], qz[7], qw[7]; qw already
// includes the panel area and 1/(4 pi).  c32/q32/q4 are coordinates relative to
// the mesh centre (`shift`), in float.  q4 holds the same float points as 7
// arrays of n (x, y, z, w) quadruples, point-major, so that one 16-byte load
// per point brings all four and consecutive panels stay contiguous.
struct Tab {
  int n;
  const double* cen;   // 3n: x[], y[], z[]
  const double* h2;    // n: squared longest edge
  const double* vert;  // 9n: v0x v0y v0z v1x ... v2z
  const double* area;  // n
  const double* q64;   // 28n
  const float* c32;    // 3n
  const float* q32;    // 28n
  const float4* q4;    // 7n: (x, y, z, w) of point a of panel p at a n + p
  const double* n64;   // 3n: unit normals nx[], ny[], nz[] ((v1 - v0) x (v2 - v0) / |.|)
  const float* n32;    // 3n: the same in float
  const Consts* K;
};

constexpr double INV4PI = 0.079577471545947667884441881686257181;

// exp(-sigma r) / r  with sigma = s / c complex, for float or double
__device__ __forceinline__ cpx<float> green(float r, float sr, float si) {
  float e = expf(-sr * r) / r;
  float sn, cs;
  sincosf(si * r, &sn, &cs);
  return {e * cs, -e * sn};
}
__device__ __forceinline__ cpx<double> green(double r, double sr, double si) {
  double e = exp(-sr * r) / r;
  double sn, cs;
  sincos(si * r, &sn, &cs);
  return {e * cs, -e * sn};
}

// far tier: 7-point rule, in T arithmetic
template <typename T>
struct FarData;
template <>
struct FarData<float> {
  static __device__ __forceinline__ const float* q(const Tab& t) { return t.q32; }
  static __device__ __forceinline__ const float* c(const Tab& t) { return t.c32; }
};
template <>
struct FarData<double> {
  static __device__ __forceinline__ const double* q(const Tab& t) { return t.q64; }
  static __device__ __forceinline__ const double* c(const Tab& t) { return t.cen; }
};

template <typename T>
__device__ __forceinline__ cpx<T> far_entry(const Tab& t, T xi, T yi, T zi, int pj, T sr, T si) {
  const T* q = FarData<T>::q(t);
  const int n = t.n;
  cpx<T> acc = {T(0), T(0)};
#pragma unroll
  for (int a = 0; a < NQ_FAR; ++a) {
    T dx = xi - q[(a)*n + pj];
    T dy = yi - q[(7 + a) * n + pj];
    T dz = zi - q[(14 + a) * n + pj];
    T w = q[(21 + a) * n + pj];
    T r = sqrt(dx * dx + dy * dy + dz * dz);
    cpx<T> g = green(r, sr, si);
    acc.re += w * g.re;
    acc.im += w * g.im;
  }
  return acc;
}

// float far tier on the hardware transcendental units: exp(-sr r) as
// 2^(-sr log2(e) r), the phase si r reduced to [-1/2, 1/2] revolutions before
// the hardware sine/cosine (which take revolutions), 1/r from the reciprocal
// square root.  The argument products carry the same float rounding as the
// generic path; the reduction is exact (subtraction of the nearest integer).
template <>
__device__ __forceinline__ cpx<float> far_entry<float>(const Tab& t, float xi, float yi, float zi,
                                                       int pj, float sr, float si) {
  const float4* q = t.q4;
  const int n = t.n;
  const float a2 = -sr * 1.44269504088896340736f;   // -sr log2(e)
  const float rv = si * 0.159154943091895335769f;   // si / (2 pi)
  float ar = 0.f, ai = 0.f;
#pragma unroll
  for (int a = 0; a < NQ_FAR; ++a) {
    const float4 qa = q[a * n + pj];
    const float dx = xi - qa.x;
    const float dy = yi - qa.y;
    const float dz = zi - qa.z;
    const float w = qa.w;
    const float r2 = dx * dx + dy * dy + dz * dz;
    const float ri = __builtin_amdgcn_rsqf(r2);
    const float r = r2 * ri;
    const float e = __builtin_amdgcn_exp2f(a2 * r) * (ri * w);
    float rev = rv * r;
    rev -= rintf(rev);
    ar += e * __builtin_amdgcn_cosf(rev);
    ai -= e * __builtin_amdgcn_sinf(rev);
  }
  return {ar, ai};
}

// near tier: 7-point rule on 16 sub-triangles, double
__device__ __forceinline__ cpx<double> near_entry(const Tab& t, int pi, int pj, double sr,
                                                   double si) {
  const int n = t.n;
  const double xi = t.cen[pi], yi = t.cen[n + pi], zi = t.cen[2 * n + pi];
  double v[9];
#pragma unroll
  for (int c = 0; c < 9; ++c) v[c] = t.vert[c * n + pj];
  const double wa = t.area[pj] * INV4PI;
  cpx<double> acc = {0.0, 0.0};
  for (int a = 0; a < NQ_NEAR; ++a) {
    const double b0 = t.K->nb[a][0], b1 = t.K->nb[a][1], b2 = t.K->nb[a][2];
    double px = b0 * v[0] + b1 * v[3] + b2 * v[6];
    double py = b0 * v[1] + b1 * v[4] + b2 * v[7];
    double pz = b0 * v[2] + b1 * v[5] + b2 * v[8];
    double dx = xi - px, dy = yi - py, dz = zi - pz;
    double r = sqrt(dx * dx + dy * dy + dz * dz);
    cpx<double> g = green(r, sr, si);
    double w = t.K->nw[a] * wa;
    acc.re += w * g.re;
    acc.im += w * g.im;
  }
  return acc;
}

// (1 - exp(-a)) / a for complex a; series below |a| = 1e-3
__device__ __forceinline__ cpx<double> phi_c(double ar, double ai) {
  double m2 = ar * ar + ai * ai;
  if (m2 < 1e-6) {
    // 1 - a/2 + a^2/6 - a^3/24
    double a2r = ar * ar - ai * ai, a2i = 2.0 * ar * ai;
    double a3r = a2r * ar - a2i * ai, a3i = a2r * ai + a2i * ar;
    return {1.0 - 0.5 * ar + a2r / 6.0 - a3r / 24.0, -0.5 * ai + a2i / 6.0 - a3i / 24.0};
  }
  double e = exp(-ar);
  double sn, cs;
  sincos(ai, &sn, &cs);
  double nr = 1.0 - e * cs, ni = e * sn;  // 1 - exp(-a)
  // (nr + i ni) / (ar + i ai)
  return {(nr * ar + ni * ai) / m2, (ni * ar - nr * ai) / m2};
}

// self tier: polar coordinates about the centroid; radial integral exact,
// angle by 16-point Gauss-Legendre over each edge's angular range
__device__ __forceinline__ cpx<double> self_entry(const Tab& t, int p, double sr, double si) {
  const int n = t.n;
  const double x[3] = {t.cen[p], t.cen[n + p], t.cen[2 * n + p]};
  double v[9];
#pragma unroll
  for (int c = 0; c < 9; ++c) v[c] = t.vert[c * n + p];
  cpx<double> acc = {0.0, 0.0};
  for (int e = 0; e < 3; ++e) {
    const double* P = v + 3 * e;
    const double* Q = v + 3 * ((e + 1) % 3);
    double ex = Q[0] - P[0], ey = Q[1] - P[1], ez = Q[2] - P[2];
    double el = sqrt(ex * ex + ey * ey + ez * ez);
    ex /= el; ey /= el; ez /= el;
    double px = P[0] - x[0], py = P[1] - x[1], pz = P[2] - x[2];
    double qx = Q[0] - x[0], qy = Q[1] - x[1], qz = Q[2] - x[2];
    double tp = px * ex + py * ey + pz * ez;
    double tq = qx * ex + qy * ey + qz * ez;
    double fx = px - tp * ex, fy = py - tp * ey, fz = pz - tp * ez;
    double d = sqrt(fx * fx + fy * fy + fz * fz);
    double ta = atan2(tp, d), tb = atan2(tq, d);
    double span = tb - ta;
    cpx<double> part = {0.0, 0.0};
    for (int g = 0; g < NGL; ++g) {
      double th = ta + span * t.K->gl_x[g];
      double R = d / cos(th);
      cpx<double> f = phi_c(sr * R, si * R);
      double w = t.K->gl_w[g] * R;
      part.re += w * f.re;
      part.im += w * f.im;
    }
    acc.re += span * part.re;
    acc.im += span * part.im;
  }
  acc.re *= INV4PI;
  acc.im *= INV4PI;
  return acc;
}

// tier decision in double on squared lengths: near iff |x_i - x_j|^2 < 4 h_j^2
__device__ __forceinline__ bool is_near(const Tab& t, int pi, int pj) {
#pragma clang fp contract(off)
  const int n = t.n;
  double dx = t.cen[pi] - t.cen[pj];
  double dy = t.cen[n + pi] - t.cen[n + pj];
  double dz = t.cen[2 * n + pi] - t.cen[2 * n + pj];
  double d2 = dx * dx + dy * dy + dz * dz;
  return d2 < 4.0 * t.h2[pj];
}

// entry at internal positions (pi, pj), frequency sigma = s / c; far tier in T.
// ALLFAR: the caller guarantees that no self/near-tier pair occurs (blocks whose
// boxes are far enough apart), so the float64 tiers are not compiled in.
template <typename T, bool ALLFAR = false>
__device__ __forceinline__ cpx<T> entry(const Tab& t, int pi, int pj, double sr, double si,
                                        bool all_far) {
  if (!ALLFAR && !all_far) {
    if (pi == pj) {
      cpx<double> e = self_entry(t, pi, sr, si);
      return {T(e.re), T(e.im)};
    }
    if (is_near(t, pi, pj)) {
      cpx<double> e = near_entry(t, pi, pj, sr, si);
      return {T(e.re), T(e.im)};
    }
  }
  const T* c = FarData<T>::c(t);
  const int n = t.n;
  return far_entry<T>(t, c[pi], c[n + pi], c[2 * n + pi], pj, T(sr), T(si));
}

// Part p of P of an entry: the far tier's quadrature points a = p, p + P, ...
// (the lanes p = 0..P-1 of an aligned group add their parts); a self or
// near-tier entry is evaluated whole by part 0.
template <typename T>
__device__ __forceinline__ cpx<T> far_entry_part(const Tab& t, T xi, T yi, T zi, int pj, T sr, T si,
                                                 int p, int P) {
  const T* q = FarData<T>::q(t);
  const int n = t.n;
  cpx<T> acc = {T(0), T(0)};
  for (int a = p; a < NQ_FAR; a += P) {
    T dx = xi - q[(a)*n + pj];
    T dy = yi - q[(7 + a) * n + pj];
    T dz = zi - q[(14 + a) * n + pj];
    T w = q[(21 + a) * n + pj];
    T r = sqrt(dx * dx + dy * dy + dz * dz);
    cpx<T> g = green(r, sr, si);
    acc.re += w * g.re;
    acc.im += w * g.im;
  }
  return acc;
}
template <>
__device__ __forceinline__ cpx<float> far_entry_part<float>(const Tab& t, float xi, float yi, float zi,
                                                            int pj, float sr, float si, int p, int P) {
  const float4* q = t.q4;
  const int n = t.n;
  const float a2 = -sr * 1.44269504088896340736f;   // -sr log2(e)
  const float rv = si * 0.159154943091895335769f;   // si / (2 pi)
  float ar = 0.f, ai = 0.f;
  for (int a = p; a < NQ_FAR; a += P) {
    const float4 qa = q[a * n + pj];
    const float dx = xi - qa.x;
    const float dy = yi - qa.y;
    const float dz = zi - qa.z;
    const float w = qa.w;
    const float r2 = dx * dx + dy * dy + dz * dz;
    const float ri = __builtin_amdgcn_rsqf(r2);
    const float r = r2 * ri;
    const float e = __builtin_amdgcn_exp2f(a2 * r) * (ri * w);
    float rev = rv * r;
    rev -= rintf(rev);
    ar += e * __builtin_amdgcn_cosf(rev);
    ai -= e * __builtin_amdgcn_sinf(rev);
  }
  return {ar, ai};
}

template <typename T, bool ALLFAR = false>
__device__ __forceinline__ cpx<T> entry_part(const Tab& t, int pi, int pj, double sr, double si,
                                             bool all_far, int p, int P) {
  if (P == 1) return entry<T, ALLFAR>(t, pi, pj, sr, si, all_far);
  if (!ALLFAR && !all_far) {
    if (pi == pj || is_near(t, pi, pj)) {
      if (p != 0) return {T(0), T(0)};
      const cpx<double> e = pi == pj ? self_entry(t, pi, sr, si) : near_entry(t, pi, pj, sr, si);
      return {T(e.re), T(e.im)};
    }
  }
  const T* c = FarData<T>::c(t);
  const int n = t.n;
  return far_entry_part<T>(t, c[pi], c[n + pi], c[2 * n + pi], pj, T(sr), T(si), p, P);
}

// ---- double layer: the normal derivative in y of exp(-sigma r) / (4 pi r) -------
// d/dn_y = (d . n_y) (1 + sigma r) exp(-sigma r) / (4 pi r^3), d = x - y; the
// 1/(4 pi) sits in the quadrature weights as for the single layer

// (1 + sigma r) exp(-sigma r) for sigma = sr + i si
__device__ __forceinline__ cpx<float> dlp_radial(float r, float sr, float si) {
  const float e = expf(-sr * r);
  float sn, cs;
  sincosf(si * r, &sn, &cs);
  const float a = 1.f + sr * r, b = si * r;
  return {e * (a * cs + b * sn), e * (b * cs - a * sn)};
}
__device__ __forceinline__ cpx<double> dlp_radial(double r, double sr, double si) {
  const double e = exp(-sr * r);
  double sn, cs;
  sincos(si * r, &sn, &cs);
  const double a = 1.0 + sr * r, b = si * r;
  return {e * (a * cs + b * sn), e * (b * cs - a * sn)};
}

// unit normal of panel p (table built with the panel tables)
template <typename T>
struct NrmData;
template <>
struct NrmData<float> {
  static __device__ __forceinline__ const float* n(const Tab& t) { return t.n32; }
};
template <>
struct NrmData<double> {
  static __device__ __forceinline__ const double* n(const Tab& t) { return t.n64; }
};
template <typename T>
__device__ __forceinline__ void panel_normal(const Tab& t, int p, T nrm[3]) {
  const T* nn = NrmData<T>::n(t);
  nrm[0] = nn[p];
  nrm[1] = nn[t.n + p];
  nrm[2] = nn[2 * t.n + p];
}

// near tier of the double layer: 112-point rule, double
__device__ __forceinline__ cpx<double> dlp_near_entry(const Tab& t, int pi, int pj, double sr, double si) {
  const int n = t.n;
  double nrm[3];
  panel_normal(t, pj, nrm);
  const double xi = t.cen[pi], yi = t.cen[n + pi], zi = t.cen[2 * n + pi];
  double v[9];
#pragma unroll
  for (int c = 0; c < 9; ++c) v[c] = t.vert[c * n + pj];
  const double wa = t.area[pj] * INV4PI;
  double ar = 0.0, ai = 0.0;
  for (int a = 0; a < NQ_NEAR; ++a) {
    const double b0 = t.K->nb[a][0], b1 = t.K->nb[a][1], b2 = t.K->nb[a][2];
    const double dx = xi - (b0 * v[0] + b1 * v[3] + b2 * v[6]);
    const double dy = yi - (b0 * v[1] + b1 * v[4] + b2 * v[7]);
    const double dz = zi - (b0 * v[2] + b1 * v[5] + b2 * v[8]);
    const double r2 = dx * dx + dy * dy + dz * dz, r = sqrt(r2);
    const double f = t.K->nw[a] * wa * (dx * nrm[0] + dy * nrm[1] + dz * nrm[2]) / (r2 * r);
    const cpx<double> g = dlp_radial(r, sr, si);
    ar += f * g.re;
    ai += f * g.im;
  }
  return {ar, ai};
}

// far tier of the double layer, quadrature points a = p, p + P, ... in T
template <typename T>
__device__ __forceinline__ cpx<T> dlp_far_entry_part(const Tab& t, int pi, int pj, T sr, T si, int p, int P) {
  const int n = t.n;
  T nrm[3];
  panel_normal(t, pj, nrm);
  const T* q = FarData<T>::q(t);
  const T* c = FarData<T>::c(t);
  const T xi = c[pi], yi = c[n + pi], zi = c[2 * n + pi];
  const T nx = nrm[0], ny = nrm[1], nz = nrm[2];
  T ar = T(0), ai = T(0);
  for (int a = p; a < NQ_FAR; a += P) {
    const T dx = xi - q[a * n + pj];
    const T dy = yi - q[(7 + a) * n + pj];
    const T dz = zi - q[(14 + a) * n + pj];
    const T w = q[(21 + a) * n + pj];
    const T r2 = dx * dx + dy * dy + dz * dz, r = sqrt(r2);
    const T f = w * (dx * nx + dy * ny + dz * nz) / (r2 * r);
    const cpx<T> g = dlp_radial(r, sr, si);
    ar += f * g.re;
    ai += f * g.im;
  }
  return {ar, ai};
}

// float far tier of the double layer on the hardware transcendental units, as
// far_entry<float>: exp(-sr r) as 2^(-sr log2(e) r), the phase reduced to
// [-1/2, 1/2] revolutions, 1/r from the reciprocal square root
template <>
__device__ __forceinline__ cpx<float> dlp_far_entry_part<float>(const Tab& t, int pi, int pj, float sr, float si,
                                                                int p, int P) {
  const int n = t.n;
  const float4* q = t.q4;
  const float xi = t.c32[pi], yi = t.c32[n + pi], zi = t.c32[2 * n + pi];
  const float nx = t.n32[pj], ny = t.n32[n + pj], nz = t.n32[2 * n + pj];
  const float a2 = -sr * 1.44269504088896340736f;   // -sr log2(e)
  const float rv = si * 0.159154943091895335769f;   // si / (2 pi)
  float ar = 0.f, ai = 0.f;
  for (int a = p; a < NQ_FAR; a += P) {
    const float4 qa = q[a * n + pj];
    const float dx = xi - qa.x;
    const float dy = yi - qa.y;
    const float dz = zi - qa.z;
    const float r2 = dx * dx + dy * dy + dz * dz;
    const float ri = __builtin_amdgcn_rsqf(r2);
    const float r = r2 * ri;
    const float f = __builtin_amdgcn_exp2f(a2 * r) * qa.w * (dx * nx + dy * ny + dz * nz) * (ri * ri * ri);
    float rev = rv * r;
    rev -= rintf(rev);
    const float cs = __builtin_amdgcn_cosf(rev), sn = __builtin_amdgcn_sinf(rev);
    const float b = 1.f + sr * r, c = si * r;
    ar += f * (b * cs + c * sn);
    ai += f * (c * cs - b * sn);
  }
  return {ar, ai};
}

// part p of P of a double-layer entry (as entry_part): self 0 (the centroid
// lies in its flat panel's plane), near tier whole by part 0 in double
template <typename T, bool ALLFAR = false>
__device__ __forceinline__ cpx<T> dlp_entry_part(const Tab& t, int pi, int pj, double sr, double si,
                                                 bool all_far, int p, int P) {
  if (!ALLFAR && !all_far) {
    if (pi == pj) return {T(0), T(0)};
    if (is_near(t, pi, pj)) {
      if (p != 0) return {T(0), T(0)};
      const cpx<double> e = dlp_near_entry(t, pi, pj, sr, si);
      return {T(e.re), T(e.im)};
    }
  }
  return dlp_far_entry_part<T>(t, pi, pj, T(sr), T(si), p, P);
}

// entry part of the single (DLP = false) or double layer
template <typename T, bool ALLFAR, bool DLP>
__device__ __forceinline__ cpx<T> op_entry_part(const Tab& t, int pi, int pj, double sr, double si,
                                                bool all_far, int p, int P) {
  if constexpr (DLP)
    return dlp_entry_part<T, ALLFAR>(t, pi, pj, sr, si, all_far, p, P);
  else
    return entry_part<T, ALLFAR>(t, pi, pj, sr, si, all_far, p, P);
}

// threadIdx.x hidden from loop-invariant code motion: address arithmetic
// derived from it stays next to its use instead of holding a register across
// an enclosing persistent loop (the empty asm emits no instruction)
__device__ __forceinline__ int opaque_tid() {
  int t = threadIdx.x;
  asm volatile("" : "+v"(t));
  return t;
}

// lanes per entry when a row of len entries is spread over nt threads: the
// largest power of two <= 8 that still gives every entry its own lanes
__device__ __forceinline__ int split_lanes(int nt, int len) {
  int P = 1;
  while (P < 8 && nt / (2 * P) >= len) P *= 2;
  return P;
}

// sum over the aligned group of P lanes (P a power of two <= 64); every lane of
// the group receives it
template <typename T>
__device__ __forceinline__ cpx<T> lanes_sum(cpx<T> v, int P) {
  for (int o = 1; o < P; o <<= 1) {
    v.re += __shfl_xor(v.re, o, WAVE);
    v.im += __shfl_xor(v.im, o, WAVE);
  }
  return v;
}

}  // namespace gcq
